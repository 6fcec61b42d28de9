"""Planted mistakes: each case alters one or two lines of a copy of the
oracle package (its C source, or the Python module that builds the graph
problems' matrices) in the way a plausible slip would (a dropped term, a
flipped sign, a wrong or transposed operand, an inverted test) and runs the
pins of tests/test_oracle_pins.py against that copy.  Every altered oracle
must fail at least one pin, which shows that the pins bind each step of the
oracle and do not merely re-run it.  CPU only; the oracle in the tree is not
touched."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "oracle")

# C source: (what the slip is, the exact text of the line, the altered text)
MUTANTS = [
    ("reuse: start not rescaled to the Algorithm 1 level",
     "double th = eps / ymax;", "double th = 1.0 / ymax;"),
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
    ("Newton: covering derivative weighted toward the largest row",
     "double t = exp(-st->eta * (st->z[j] + alpha * st->dz[j] - zmn));",
     "double t = exp(st->eta * (st->z[j] + alpha * st->dz[j] - zmn));"),
    ("Newton: quotient rule with the wrong sign",
     "double gp = (e.psi * dphi - e.phi * dpsi) / (e.psi * e.psi);",
     "double gp = (e.psi * dphi + e.phi * dpsi) / (e.psi * e.psi);"),
    ("Newton: step taken against the correction",
     "next = a - corr;", "next = a + corr;"),
    ("Newton: iterates not kept inside the bracket",
     "if (!(next > lo && next < hi)) {", "if (!(next == next)) {"),
    ("drop: met rows kept in the smoothed minimum",
     "if (st->z[j] < 1.0) { st->ai[st->na] = j;", "if (st->z[j] < 2.0) { st->ai[st->na] = j;"),
    ("drop: weights of met rows left in u",
     "for (int64_t j = 0; j < st->mC; ++j) st->u[j] = 0.0;", "for (int64_t j = 0; j < 0; ++j) st->u[j] = 0.0;"),
    ("mixed optimization: objective row scaled by M instead of 1/M",
     "for (int64_t i = 0; i < n; ++i) val[nnz + i] = c[i] / M;", "for (int64_t i = 0; i < n; ++i) val[nnz + i] = c[i] * M;"),
    ("mixed optimization: a feasible minimization probe moves the lower end",
     "else { if (M < hi) hi = M; shi = M; }", "else { if (M > lo) lo = M; shi = M; }"),
    ("level sets: edge counted at its first endpoint",
     "cnt[(a > b ? a : b) + 1]++;", "cnt[(a < b ? a : b) + 1]++;"),
]


# Python matrix builders (Section 3 formulations)
PY_MUTANTS = [
    ("dominating set: identity left out of I + A",
     "    r = np.concatenate([g.u, g.v, ar])\n    c = np.concatenate([g.v, g.u, ar])",
     "    r = np.concatenate([g.u, g.v])\n    c = np.concatenate([g.v, g.u])"),
    ("dominating set: A taken one way only",
     "    r = np.concatenate([g.u, g.v, ar])\n    c = np.concatenate([g.v, g.u, ar])",
     "    r = np.concatenate([g.u, ar])\n    c = np.concatenate([g.v, ar])"),
    ("incidence: second endpoint replaced by the first",
     "np.concatenate([u, v]), np.concatenate([e, e]))", "np.concatenate([u, u]), np.concatenate([e, e]))"),
    ("vertex cover: edge rows hold one endpoint twice",
     "np.concatenate([newid[g.u], newid[g.v]]))", "np.concatenate([newid[g.u], newid[g.u]]))"),
    ("densest: W rows cover one orientation twice",
     "W = CSR.from_coo(m, 2 * m, np.concatenate([e, e]), np.concatenate([2 * e, 2 * e + 1]))",
     "W = CSR.from_coo(m, 2 * m, np.concatenate([e, e]), np.concatenate([2 * e, 2 * e]))"),
    ("packing normalisation: objective weights dropped",
     "A.val / (b[rows] * c[A.idx])", "A.val / b[rows]"),
]

CASES = [("mwu_oracle.c",) + m for m in MUTANTS] + [("__init__.py",) + m for m in PY_MUTANTS]


@pytest.mark.parametrize("fname,what,old,new", CASES, ids=[c[1] for c in CASES])
def test_planted_mistake_fails_a_pin(tmp_path, fname, what, old, new):
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    for f in ("mwu_oracle.c", "__init__.py"):
        shutil.copy(os.path.join(PKG, f), pkg / f)
    text = (pkg / fname).read_text()
    assert text.count(old) == 1, f"mutation site not unique or missing: {old!r}"
    (pkg / fname).write_text(text.replace(old, new))
    env = dict(os.environ, ORACLE_PKG_OVERRIDE=str(tmp_path))
    p = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    tail = "\n".join(p.stdout.splitlines()[-3:])
    # 1: a pin failed (0 would mean the mistake went unnoticed)
    assert p.returncode == 1, f"{what}: pytest exit {p.returncode}\n{tail}"


def test_unaltered_copy_passes(tmp_path):
    """The harness itself: the copied package, unaltered, passes every pin,
    so each failure above comes from its planted slip."""
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    for f in ("mwu_oracle.c", "__init__.py"):
        shutil.copy(os.path.join(PKG, f), pkg / f)
    env = dict(os.environ, ORACLE_PKG_OVERRIDE=str(tmp_path))
    code = ("import sys, os; sys.path.insert(0, os.environ['ORACLE_PKG_OVERRIDE']); import oracle; "
            "print(oracle.__file__)")
    where = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           check=True).stdout.strip()
    assert where == str(pkg / "__init__.py")
    p = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        "-q", "-p", "no:cacheprovider", "-m", "not gpu"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert p.returncode == 0, p.stdout[-2000:]
    assert (pkg / "libmwu_oracle.so").exists()        # the pins ran against the copy
