"""Planted mistakes in the oracle must each fail at least one pin.

Every case copies oracle.c, makes one plausible mistake by a textual
substitution, compiles the copy with gcc into a temporary library and runs the
pins on it.  Nothing here touches the GPU library.
"""
import os
import subprocess
import sys

import pytest

from oracle import build as obuild
from tests import oracle_pins

SRC = open(obuild.SRC).read()

MUTANTS = {
    "product operand order": ("s += A[a * 3 + k] * B[k * 3 + b];", "s += B[a * 3 + k] * A[k * 3 + b];"),
    "product neighbour -mu": ("shifted(L, x, y, z, mu, 1, &xs, &ys, &zs);\n                        const cplx *A",
                              "shifted(L, x, y, z, mu, -1, &xs, &ys, &zs);\n                        const cplx *A"),
    "product transposed": ("s += A[a * 3 + k] * B[k * 3 + b];", "s += A[k * 3 + a] * B[b * 3 + k];"),
    "laplacian quarter dropped": ("o[c] = 0.25 * acc[c];", "o[c] = acc[c];"),
    "laplacian -6 dropped": ("acc[c] = -6.0 * here[c];", "acc[c] = -4.0 * here[c];"),
    "laplacian one-site hop": ("shifted(L, x, y, z, mu, 2, &xs, &ys, &zs);", "shifted(L, x, y, z, mu, 1, &xs, &ys, &zs);"),
    "laplacian backward no dagger": ("matvec_dag(twolink(L, W, xs, ys, zs, t, mu)", "matvec(twolink(L, W, xs, ys, zs, t, mu)"),
    "laplacian backward link at x": ("matvec_dag(twolink(L, W, xs, ys, zs, t, mu), in", "matvec_dag(twolink(L, W, x, y, z, t, mu), in"),
    "laplacian forward dagger": ("matvec(twolink(L, W, x, y, z, t, mu)", "matvec_dag(twolink(L, W, x, y, z, t, mu)"),
    "dagger is transpose": ("s += conj(M[b * 3 + a]) * v[b];", "s += M[b * 3 + a] * v[b];"),
    "matvec transposed": ("s += M[a * 3 + b] * v[b];", "s += M[b * 3 + a] * v[b];"),
    "second form reversed order": ("matvec(link(L, U, x, y, z, t, mu), src", "matvec(link(L, U, xs, ys, zs, t, mu), src"),
    "second form sign": ("out[i] += chi2[i];", "out[i] -= chi2[i];"),
    "smear step sigma": ("double step = sigma / (double)n;", "double step = sigma;"),
    "smear one step short": ("for (int k = 0; k < n; k++) {\n        or_lap_twolink", "for (int k = 1; k < n; k++) {\n        or_lap_twolink"),
    "smear wrong slice": ("or_smear(L, W, t_of_rhs[r], n, sigma", "or_smear(L, W, 0, n, sigma"),
    "onelink hop two sites": ("shifted(L, x, y, z, mu, 1, &xs, &ys, &zs);\n                    matvec(link(",
                              "shifted(L, x, y, z, mu, 2, &xs, &ys, &zs);\n                    matvec(link("),
    "onelink hop forward link at neighbour": ("matvec(link(L, U, x, y, z, t, mu), in + site3(L, xs, ys, zs) * 3, tmp);",
                                              "matvec(link(L, U, xs, ys, zs, t, mu), in + site3(L, xs, ys, zs) * 3, tmp);"),
    "onelink laplacian centre -1": ("acc[a] += f[a] - 2.0 * c[a] + b[a];", "acc[a] += f[a] - 1.0 * c[a] + b[a];"),
    "onelink laplacian backward no dagger": ("matvec_dag(link(L, U, xb, yb, zb, t, mu)", "matvec(link(L, U, xb, yb, zb, t, mu)"),
    "onelink laplacian backward link at x": ("matvec_dag(link(L, U, xb, yb, zb, t, mu)", "matvec_dag(link(L, U, x, y, z, t, mu)"),
    "gsmear alpha sign": ("psi[i] += alpha * h[i];", "psi[i] -= alpha * h[i];"),
    "onelink smear one step short": ("for (int k = 0; k < n; k++) {\n        or_lap_onelink",
                                     "for (int k = 1; k < n; k++) {\n        or_lap_onelink"),
    "norm drops imaginary": ("s += creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);", "s += creal(psi[i]) * creal(psi[i]);"),
    "dot conjugates second": ("s += conj(phi[i]) * psi[i];", "s += phi[i] * conj(psi[i]);"),
    "site norm no sqrt": ("out[i] = sqrt(s);", "out[i] = s;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    assert SRC.count(old) >= 1, f"mutation anchor not found: {old!r}"
    src = tmp_path / "oracle_mutant.c"
    src.write_text(SRC.replace(old, new, 1))
    lib = str(tmp_path / "liboracle_mutant.so")
    obuild.build(str(src), lib)
    code = (
        "import sys\n"
        f"sys.path.insert(0, {os.path.dirname(os.path.dirname(os.path.abspath(__file__)))!r})\n"
        "from oracle.core import Oracle\n"
        "from tests import oracle_pins\n"
        f"o = Oracle({lib!r})\n"
        "failed = []\n"
        "for p in oracle_pins.ALL_PINS:\n"
        "    try:\n"
        "        p(o)\n"
        "    except AssertionError:\n"
        "        failed.append(p.__name__)\n"
        "print(','.join(failed))\n"
    )
    # a subprocess keeps a mutant that crashes (bad index) from taking the test run down
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    caught = res.returncode != 0 or res.stdout.strip() != ""
    assert caught, f"mutant '{name}' passed every pin"
