"""The pins catch plausible mistakes in the checker.

Each case plants one mistake in a copy of the checker's C source (or, for
the optimiser, in its Python reference), builds it on the CPU and runs the
pin that is meant to catch it against the mutant: the pin must fail.  The
unmodified checker passes the same pins in test_oracle_pins.py.
"""

import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "geer_oracle.c")
PINS = "tests/test_oracle_pins.py"

# (name, [(text, replacement), ...], pins that must fail)
MUTATIONS = [
    ("ell one too long (Eq. ell without the -1)",
     [("/ log(1.0 / lambda) - 1.0;\n    double c = ceil(v);\n    if (c < 0.0) return 0;\n    return (int32_t)c;\n}\n\n/* Eq. (old-ell)",
       "/ log(1.0 / lambda);\n    double c = ceil(v);\n    if (c < 0.0) return 0;\n    return (int32_t)c;\n}\n\n/* Eq. (old-ell)")],
     ["test_ell_is_smallest_length_meeting_the_tail_bound"]),
    ("old-ell one too long",
     [("double v = log(4.0 / (eps - eps * lambda)) / log(1.0 / lambda) - 1.0;",
       "double v = log(4.0 / (eps - eps * lambda)) / log(1.0 / lambda);")],
     ["test_peng_ell_is_smallest_length_meeting_its_bound"]),
    ("psi with ceil and floor swapped (Eq. Delta-st)",
     [("double up = (double)((lf + 1) / 2);\n    double dn = (double)(lf / 2);",
       "double up = (double)(lf / 2);\n    double dn = (double)((lf + 1) / 2);")],
     ["test_psi_is_attained_by_an_alternating_walk"]),
    ("psi too large (max1 counted at every position)",
     [("double up = (double)((lf + 1) / 2);\n    double dn = (double)(lf / 2);",
       "double up = (double)lf;\n    double dn = (double)(lf / 2);")],
     ["test_psi_is_attained_by_an_alternating_walk"]),
    ("Bernstein width without the factor 2 under the root (Eq. fx)",
     [("return sqrt(2.0 * var * lg / nz) + 3.0 * psi * lg / nz;",
       "return sqrt(var * lg / nz) + 3.0 * psi * lg / nz;")],
     ["test_bernstein_width_brackets_the_normal_quantile"]),
    ("Bernstein width without the square root",
     [("return sqrt(2.0 * var * lg / nz) + 3.0 * psi * lg / nz;",
       "return 2.0 * var * lg / nz + 3.0 * psi * lg / nz;")],
     ["test_bernstein_width_brackets_the_normal_quantile"]),
    ("Bernstein width without its range term",
     [("return sqrt(2.0 * var * lg / nz) + 3.0 * psi * lg / nz;",
       "return sqrt(2.0 * var * lg / nz);")],
     ["test_bernstein_width_covers_the_mean_on_small_samples"]),
    ("greedy switch stops one hop late",
     [("    int64_t supp_sum = support_degree_sum(n, rp, sx) + support_degree_sum(n, rp, sy);\n    if (ell > 0 && target > 0) {",
       "    int64_t supp_sum = support_degree_sum(n, rp, sx) + support_degree_sum(n, rp, sy);\n    int late = 0;\n    if (ell > 0 && target > 0) {"),
      ("if ((double)supp_sum > h) break;",
       "if ((double)supp_sum > h) { if (late) break; late = 1; }")],
     ["test_greedy_switch_stops_at_the_first_hop_where_the_rule_holds"]),
    ("greedy switch stops one hop early (rule at half the budget)",
     [("if ((double)supp_sum > h) break;", "if ((double)supp_sum > 0.5 * h) break;")],
     ["test_greedy_switch_stops_at_the_first_hop_where_the_rule_holds"]),
]


def _build_mutant(tmp_path, edits):
    src = open(SRC).read()
    for old, new in edits:
        assert src.count(old) == 1, f"mutation anchor not found once: {old[:60]!r}"
        src = src.replace(old, new)
    c = tmp_path / "mutant.c"
    c.write_text(src)
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", str(so), str(c),
                           "-lm", "-lpthread"])
    return str(so)


@pytest.mark.parametrize("name,edits,pins", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pin_catches_planted_mistake(tmp_path, name, edits, pins):
    so = _build_mutant(tmp_path, edits)
    env = dict(os.environ, GEER_ORACLE_LIB=so)
    for pin in pins:
        res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                              f"{PINS}::{pin}"], cwd=ROOT, env=env, capture_output=True,
                             text=True, timeout=600)
        assert res.returncode == 1, f"{pin} did not catch: {name}\n{res.stdout[-2000:]}"
        assert " failed" in res.stdout, res.stdout[-2000:]


def test_pin_catches_adam_without_bias_correction(monkeypatch):
    from oracle import mlp

    import test_oracle_pins as pins

    def adam_no_correction(p, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        m = beta1 * m + (1 - beta1) * g
        v = beta2 * v + (1 - beta2) * g * g
        return p - lr * m / (np.sqrt(v) + eps), m, v

    monkeypatch.setattr(mlp, "adam_step", adam_no_correction)
    with pytest.raises(AssertionError):
        pins.test_mlp_reference_adam_steps_by_lr_with_bias_correction()
