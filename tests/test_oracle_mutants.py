"""Planted mistakes: each case alters one line of a copy of the oracle's C
source in the way a plausible slip would (a dropped term, a flipped sign, a
wrong or transposed operand, an inverted test) and runs the pins of
tests/test_oracle_pins.py against that copy.  Every altered oracle must fail
at least one pin, which shows that the pins bind each step of the oracle and
do not merely re-run it.  CPU only; the oracle in the tree is not touched."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mwu_oracle.c")

# (what the slip is, the exact text of the line, the altered text)
MUTANTS = [
    ("smax: max shift dropped from the value",
     "return ymax + log(sum) / eta;", "return log(sum) / eta;"),
    ("smin: wrong sign of the log term",
     "return zmin - log(sum) / eta;", "return zmin + log(sum) / eta;"),
    ("smax gradient: max shift dropped from the weights",
     "grad[i] = exp(eta * (y[i] - ymax)) / sum;", "grad[i] = exp(eta * y[i]) / sum;"),
    ("transpose product: row weight indexed by column",
     "g[A->idx[k]] += A->val[k] * w[r];", "g[A->idx[k]] += A->val[k] * w[A->idx[k] % A->rows];"),
    ("forward product: scale not applied",
     "y[r] = s * acc;", "y[r] = acc;"),
    ("Psi: wrong sign of the step",
     "s += w[i] * expm1(ea * dy[i]);", "s += w[i] * expm1(-ea * dy[i]);"),
    ("Phi: gradient weight dropped",
     "s += u[j] * expm1(-ea * dz[j]);", "s += expm1(-ea * dz[j]);"),
    ("step test inverted",
     "e.pass = (e.phi >= e.psi);", "e.pass = (e.phi <= e.psi);"),
    ("bisection keeps the wrong half",
     "if (eb.pass) lb = beta; else ub = beta;", "if (eb.pass) ub = beta; else lb = beta;"),
    ("early return of the step search dropped",
     "if (e.zmin_new >= 1.0) return alpha;          /* early return (R2) */", ""),
    ("direction: ratio transposed",
     "double r = 1.0 - st->g[i] / st->h[i];", "double r = 1.0 - st->h[i] / st->g[i];"),
    ("direction: x factor dropped",
     "di = st->step * (r > 0.0 ? r : 0.0) * st->x[i];", "di = st->step * (r > 0.0 ? r : 0.0);"),
    ("eta: covering rows left out of m",
     "st->eta = 10.0 * log((double)(st->mP + st->mC)) / eps;",
     "st->eta = 10.0 * log((double)(st->mP + 1)) / eps;"),
    ("step factor of the single-row case swapped",
     "double s = (st->mP == 1 || st->mC == 1) ? 1.0 : 0.5;",
     "double s = (st->mP == 1 || st->mC == 1) ? 0.5 : 1.0;"),
    ("initial point: column maximum dropped",
     "x[i] = eps / ((double)P->cols * cm[i]);", "x[i] = eps / ((double)P->cols);"),
    ("covering target taken as 1 + eps",
     "if (zmin >= 1.0) { res->status = ORC_FEASIBLE; break; }",
     "if (zmin >= 1.0 + eps) { res->status = ORC_FEASIBLE; break; }"),
    ("packing bound from the largest g",
     "if (st.g[i] < gmin) gmin = st.g[i];", "if (st.g[i] > gmin || gmin == INFINITY) gmin = st.g[i];"),
    ("Psi, large-step form: wrong sign of the log term",
     "return (ymx - L) + log(s) / eta;", "return (ymx - L) - log(s) / eta;"),
    ("Phi, large-step form: wrong sign of the log term",
     "return (zpm - L) - log(t) / eta;", "return (zpm - L) + log(t) / eta;"),
    ("covering bound from the smallest h",
     "if (st.h[i] > hmax) hmax = st.h[i];", "if (st.h[i] < hmax || hmax == 0.0) hmax = st.h[i];"),
    ("warm search: early return of the downward branch dropped",
     "if (eb.zmin_new >= 1.0) return b;", ""),
    ("densest: covering minimum taken as the maximum",
     "if (cov[e] < cmin) cmin = cov[e];", "if (cov[e] > cmin || cmin == INFINITY) cmin = cov[e];"),
    ("densest: returned point not rescaled",
     "z_best[i] = z[i] / cmin;", "z_best[i] = z[i];"),
    ("level sets: edge counted at its first endpoint",
     "cnt[(a > b ? a : b) + 1]++;", "cnt[(a < b ? a : b) + 1]++;"),
]


@pytest.mark.parametrize("what,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(tmp_path, what, old, new):
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site not unique or missing: {old!r}"
    src = tmp_path / "mwu_oracle.c"
    src.write_text(text.replace(old, new))
    env = dict(os.environ, ORACLE_SRC_OVERRIDE=str(src))
    p = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = "\n".join(p.stdout.splitlines()[-3:])
    # 1: a pin failed (0 would mean the mistake went unnoticed)
    assert p.returncode == 1, f"{what}: pytest exit {p.returncode}\n{tail}"
