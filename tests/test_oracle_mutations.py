"""Planted mistakes in the oracle are caught by its pins.

Each case changes one token of oracle/pv_oracle.c (a dropped term, a wrong
sign, index or factor, a transposed operand, a flipped comparison), builds
that copy with the oracle's own compiler flags into a temporary directory and
runs the pin suite (tests/test_oracle_pins.py) against it in a child process.
Every mutant must make at least one pin fail; the unmodified source must pass.
Everything runs on the CPU.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(ROOT, "oracle", "pv_oracle.c")

# (what is wrong, text in the source, replacement); each text occurs once
MUTANTS = [
    ("Eq. 1: sign of the y term", "add32(mul32(dtx, dx), mul32(dty, dy))", "sub32(mul32(dtx, dx), mul32(dty, dy))"),
    ("Eq. 3: variance over the numerator", "const float s2 = div32(vxx, den);", "const float s2 = div32(vxx, add32(den, den));"),
    ("cubic kernel: 3/4 coefficient", "sub32(0.75f, mul32(0.25f", "sub32(0.74f, mul32(0.25f"),
    ("histogram: last edge not full", "(j + 1 == nb) ? full", "(j + 1 == nb) ? 0"),
    ("argmax: last index on ties", "        if (h[j] > h[i])\n            i = j;", "        if (h[j] >= h[i])\n            i = j;"),
    ("Eq. 5: sign of delta", "0.5 * (Np - Nm) / den", "0.5 * (Nm - Np) / den"),
    ("partition point rounded up", "(a->hi + cl[live[k + 1]].lo) / 2", "(a->hi + cl[live[k + 1]].lo + 1) / 2"),
    ("removal: highest z on ties", "a->n_assoc < cl[worst].n_assoc", "a->n_assoc <= cl[worst].n_assoc"),
    ("Eq. 17: Tukey weight not squared", "return t * t;", "return t;"),
    ("Eq. 2: factor 2 of the cross term", "+ 2.0 * dz * (double)trk[6][i]", "+ dz * (double)trk[6][i]"),
    ("Eq. 9: sign of the extrapolation", "(alpha[2] - z) * tx", "(z - alpha[2]) * tx"),
    ("Eq. 8: transposed slope in H", "{{-1.0, 0.0, (double)trk[3][i]}", "{{-1.0, 0.0, (double)trk[4][i]}"),
    ("Eq. 16: factor of the predicted change", "0.5 * (d[0] * grad[0]", "1.0 * (d[0] * grad[0]"),
    ("Eq. 14: covariance from the full Hessian", "half[a][b] = 0.5 * hess_last", "half[a][b] = 1.0 * hess_last"),
    ("selection: beamline distance reversed",
     "keep = sqrt(bx * bx + by * by) <= p->max_rho_pp;", "keep = sqrt(bx * bx + by * by) >= p->max_rho_pp;"),
    ("selection: regions swapped",
     "int keep = !bad && cl[q].n_assoc >= (gas ? p->pv_min_gas : p->pv_min_pp);",
     "int keep = !bad && cl[q].n_assoc >= (gas ? p->pv_min_pp : p->pv_min_gas);"),
    ("ndof = 2 sum w - 2", "2.0 * sumw - 3.0", "2.0 * sumw - 2.0"),
    ("convergence: dz test inclusive of 10x", "below2 = q2 < tz", "below2 = q2 < 10.0 * tz"),
    ("Eq. 18: outlier term exp(-chi2_max)", "exp(-0.5 * chi2_max)", "exp(-chi2_max)"),
    ("pre-cut: V_x of Eq. 2 without the cross term",
     "+ 2.0 * dz * (double)ev[6][i]", "+ 0.0 * dz * (double)ev[6][i]"),
    ("pre-cut: seed without the beamline tilt",
     "seed[3] = {(double)beam[0] + (double)beam[2] * zs", "seed[3] = {(double)beam[0] + (double)beam[2] * 0.0"),
    ("pre-cut: y residual dropped", "const double ry = y + dz * ty - seed[1];", "const double ry = 0.0 * (y + dz * ty - seed[1]);"),
    ("duplicates: distance not squared", "if (d * d < lim)", "if (fabs(d) < lim)"),
]


def _run_pins(lib_path):
    env = dict(os.environ, PV_ORACLE_LIB=lib_path, OMP_NUM_THREADS="2")
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
           os.path.join(HERE, "test_oracle_pins.py")]
    return subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def _build_and_run(tmp, k, text):
    src = os.path.join(tmp, f"mutant{k}.c")
    with open(src, "w") as f:
        f.write(text)
    lib = oracle.build(force=True, src=src, out=os.path.join(tmp, f"libmutant{k}.so"))
    return _run_pins(lib)


def test_unmodified_oracle_passes_and_every_planted_mistake_is_caught():
    with open(SRC) as f:
        base = f.read()
    texts = []
    for what, old, new in MUTANTS:
        assert base.count(old) == 1, f"mutation site not unique or missing: {what}"
        texts.append(base.replace(old, new))
    with tempfile.TemporaryDirectory() as tmp:
        with ThreadPoolExecutor(max_workers=4) as pool:
            ref = pool.submit(_build_and_run, tmp, "ref", base)
            runs = [pool.submit(_build_and_run, tmp, k, t) for k, t in enumerate(texts)]
            r0 = ref.result()
            assert r0.returncode == 0, "unmodified oracle fails its pins:\n" + r0.stdout[-2000:]
            survivors = [MUTANTS[k][0] for k, r in enumerate(runs) if r.result().returncode == 0]
    assert not survivors, f"planted mistakes no pin catches: {survivors}"


if __name__ == "__main__":
    sys.exit(pytest.main([__file__, "-q"]))
