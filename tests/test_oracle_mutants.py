"""The pins have teeth: plausible mistakes planted in a copy of the oracle (on the
CPU) must each make at least one of its pins fail."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "vesnet_oracle.c")

# (name, original text, planted mistake) -- each original occurs in the forward sum
MUTANTS = [
    ("log sign", "ax += (long double)(w[j] * (-lnr * fx[j]", "ax += (long double)(w[j] * (+lnr * fx[j]"),
    ("dropped rr-term", "ax += (long double)(w[j] * (-lnr * fx[j] + rdotf * rx / r2",
     "ax += (long double)(w[j] * (-lnr * fx[j] + 0.0 * rdotf * rx / r2"),
    ("rr-term component swap", "ay += (long double)(w[j] * (-lnr * fy[j] + rdotf * ry / r2",
     "ay += (long double)(w[j] * (-lnr * fy[j] + rdotf * rx / r2"),
    ("ln|r| taken as ln|r|^2", "const double lnr = 0.5 * log(r2);\n            const double rdotf = rx * fx[j]",
     "const double lnr = log(r2);\n            const double rdotf = rx * fx[j]"),
    ("prefactor 1/(8 pi mu)", "const double c = 1.0 / (4.0 * VO_PI * mu);\n    int bad = 0;\n#pragma omp parallel for schedule(dynamic, 4) reduction(|:bad)\n    for (int64_t k = 0; k < n_sel; ++k) {\n        const int64_t i = sel[k];\n        long double ax = 0.0L, ay = 0.0L;\n        for (int64_t j = 0; j < n_src; ++j) {\n            if (s_ves[j] == t_excl[i]) continue;\n            const double rx = tx[i] - sx[j];\n            const double ry = ty[i] - sy[j];\n            const double r2",
     "const double c = 1.0 / (8.0 * VO_PI * mu);\n    int bad = 0;\n#pragma omp parallel for schedule(dynamic, 4) reduction(|:bad)\n    for (int64_t k = 0; k < n_sel; ++k) {\n        const int64_t i = sel[k];\n        long double ax = 0.0L, ay = 0.0L;\n        for (int64_t j = 0; j < n_src; ++j) {\n            if (s_ves[j] == t_excl[i]) continue;\n            const double rx = tx[i] - sx[j];\n            const double ry = ty[i] - sy[j];\n            const double r2"),
    ("weights dropped", "ax += (long double)(w[j] * (-lnr", "ax += (long double)(1.0 * (-lnr"),
    ("wrong vesicle excluded", "if (s_ves[j] == t_excl[i]) continue;\n            const double rx = tx[i] - sx[j];\n            const double ry = ty[i] - sy[j];\n            const double r2 = rx * rx + ry * ry;\n            if (r2 == 0.0) { bad = 1; continue; }\n            const double lnr = 0.5",
     "if (s_ves[j] == t_excl[i] + 1) continue;\n            const double rx = tx[i] - sx[j];\n            const double ry = ty[i] - sy[j];\n            const double r2 = rx * rx + ry * ry;\n            if (r2 == 0.0) { bad = 1; continue; }\n            const double lnr = 0.5"),
]


# planted in the analytic gradient: caught by the central-difference and complex-step pins
GRAD_MUTANTS = [
    ("gradient: sign of the r r^T term", "- 2.0 * gr * rF * rx / (r2 * r2);", "+ 2.0 * gr * rF * rx / (r2 * r2);"),
    ("gradient: dropped (g.F) term", "*ox = -gF * rx / r2 + (gx * rF", "*ox = 0.0 * gF * rx / r2 + (gx * rF"),
    ("gradient: dL/dw without f", "grad_w[k] = fx[j] * v_x + fy[j] * v_y;", "grad_w[k] = v_x + v_y;"),
]


def _run_pins(tmp_path, orig, bad, select):
    src = open(SRC).read()
    assert src.count(orig) == 1, f"mutation anchor {orig!r} not unique"
    mutant = tmp_path / "mutant.c"
    mutant.write_text(src.replace(orig, bad))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", str(lib), str(mutant), "-lm"])
    env = dict(os.environ, VESNET_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    return subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                           os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", select],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


@pytest.mark.parametrize("name,orig,bad", GRAD_MUTANTS, ids=[m[0] for m in GRAD_MUTANTS])
def test_planted_gradient_mistake_is_caught(tmp_path, name, orig, bad):
    r = _run_pins(tmp_path, orig, bad, "gradient or adjoint")
    assert r.returncode != 0, f"no pin caught the planted mistake {name!r}:\n{r.stdout[-2000:]}"


@pytest.mark.parametrize("name,orig,bad", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, name, orig, bad):
    src = open(SRC).read()
    assert src.count(orig) == 1, f"mutation anchor for {name!r} not unique"
    mutant = tmp_path / "mutant.c"
    mutant.write_text(src.replace(orig, bad))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99", "-o", str(lib), str(mutant), "-lm"])
    env = dict(os.environ, VESNET_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"), "-k", "not gradient and not adjoint"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"no pin caught the planted mistake {name!r}:\n{r.stdout[-2000:]}"


# planted in the Python oracles: (name, module, original text, mistake, pin file)
PY_MUTANTS = [
    ("layers: inward normal", "nearfield_rbf.py", "normal = s * np.stack([t[1], -t[0]])",
     "normal = -s * np.stack([t[1], -t[0]])", "test_oracle_rbf.py"),
    ("layers: orientation ignored", "nearfield_rbf.py", "s = 1.0 if area >= 0.0 else -1.0", "s = 1.0",
     "test_oracle_rbf.py"),
    ("layers: h as the perimeter", "nearfield_rbf.py", "h = w.sum() / n", "h = w.sum()", "test_oracle_rbf.py"),
    ("layers: reversed order", "nearfield_rbf.py", "LAYER_OFFSETS = (-1.0, -0.5, 0.0, 0.5, 1.0)",
     "LAYER_OFFSETS = (1.0, 0.5, 0.0, -0.5, -1.0)", "test_oracle_rbf.py"),
    ("rbf: width not squared", "nearfield_rbf.py", "np.exp(-r2 / (width * width))", "np.exp(-r2 / width)",
     "test_oracle_rbf.py"),
    ("rbf: back substitution with L", "nearfield_rbf.py", "solve_triangular(L.T, y, lower=False)",
     "solve_triangular(L, y, lower=True)", "test_oracle_rbf.py"),
    ("rbf: pairs not accumulated", "nearfield_rbf.py", "out[:, i] += vesicle_eval", "out[:, i] = vesicle_eval",
     "test_oracle_rbf.py"),
    ("treecode: log term sign", "treecode.py", "logpart = -MF[..., 0] * np.log(np.abs(w))",
     "logpart = MF[..., 0] * np.log(np.abs(w))", "test_oracle_treecode.py"),
    ("treecode: series index off by one", "treecode.py", "np.sum(MF[..., 1:] / k * tk[..., 1:p + 1], axis=-1)",
     "np.sum(MF[..., 1:] / (k + 1) * tk[..., 1:p + 1], axis=-1)", "test_oracle_treecode.py"),
    ("treecode: Psi not conjugated", "treecode.py", "0.5 * (w * np.conj(Phi) - np.conj(Psi))",
     "0.5 * (w * np.conj(Phi) - Psi)", "test_oracle_treecode.py"),
    ("treecode: dropped constant term", "treecode.py", "series + 0.5 * MF[..., 0] + 0.5",
     "series + 0.5", "test_oracle_treecode.py"),
    ("treecode: conj(zeta) taken about the origin", "treecode.py",
     "MPsi = box_moments(z, np.conj(zeta) * F,", "MPsi = box_moments(z, np.conj(z) * F,", "test_oracle_treecode.py"),
    ("treecode: adjacent boxes in the interaction list", "treecode.py",
     "((np.abs(sx - bx) > 1) | (np.abs(sy - by) > 1))\n            ok &= target",
     "((np.abs(sx - bx) > 0) | (np.abs(sy - by) > 0))\n            ok &= target", "test_oracle_treecode.py"),
    ("treecode: own vesicle not subtracted", "treecode.py", "u[a:b] -= direct_terms(", "u[a:b] += 0 * direct_terms(",
     "test_oracle_treecode.py"),
    ("fmm: Taylor sign of the inverse powers dropped", "fmm.py", "out[:, l] = (-1.0) ** l * np.sum(",
     "out[:, l] = np.sum(", "test_oracle_fmm.py"),
    ("fmm: binomial index off by one", "fmm.py", "float(comb(mm + l - 1, l))", "float(comb(mm + l, l))",
     "test_oracle_fmm.py"),
    ("fmm: log coefficient sign", "fmm.py", "lam * (-1.0) ** (l - 1) * Dinv ** l / l",
     "lam * (-1.0) ** l * Dinv ** l / l", "test_oracle_fmm.py"),
    ("fmm: G moments about the box centre", "fmm.py", "MG = box_moments(z, np.conj(z) * F,",
     "MG = box_moments(z, np.conj(z - centers[box]) * F,", "test_oracle_fmm.py"),
    ("fmm: constant term dropped", "fmm.py", " + 0.5 * K[row]", "", "test_oracle_fmm.py"),
    ("fmm: Phi paired with the offset from the box centre", "fmm.py", "0.5 * z[idx] * np.conj(Pv)",
     "0.5 * zeta * np.conj(Pv)", "test_oracle_fmm.py"),
    ("fmm: Q not conjugated", "fmm.py", "- 0.5 * np.conj(Qv)", "- 0.5 * Qv", "test_oracle_fmm.py"),
    ("spectral: derivative sign", "spectral.py", "1j * k * np.fft.fft(v", "-1j * k * np.fft.fft(v",
     "test_oracle_spectral.py"),
    ("spectral: tension without 1/J", "spectral.py", "tension = spectral_derivative(sigma * xs) / J",
     "tension = spectral_derivative(sigma * xs)", "test_oracle_spectral.py"),
    ("spectral: weights without 2 pi / N", "spectral.py", "J * (2.0 * np.pi / n)", "J",
     "test_oracle_spectral.py"),
]
# Not listed: keeping the even-N Nyquist wavenumber in the spectral derivative.  For real
# samples that mode's coefficient is real, so its derivative is purely imaginary and the real
# part taken at the end drops it: the change leaves every output as it was.


@pytest.mark.parametrize("name,module,orig,bad,pins", PY_MUTANTS, ids=[m[0] for m in PY_MUTANTS])
def test_planted_python_oracle_mistake_is_caught(tmp_path, name, module, orig, bad, pins):
    pkg = tmp_path / "oracle"
    pkg.mkdir()
    for f in ("__init__.py", "spectral.py", "nearfield_rbf.py", "treecode.py", "fmm.py", "oracle.py", "vesnet_oracle.c",
              "libvesnet_oracle.so"):
        if os.path.exists(os.path.join(ROOT, "oracle", f)):
            shutil.copy2(os.path.join(ROOT, "oracle", f), pkg / f)  # keeps mtimes: no rebuild of the C oracle
    src = (pkg / module).read_text()
    assert src.count(orig) == 1, f"mutation anchor for {name!r} not unique"
    (pkg / module).write_text(src.replace(orig, bad))
    env = dict(os.environ, VESNET_ORACLE_PY_ROOT=str(tmp_path))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", pins)], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode != 0, f"no pin caught the planted mistake {name!r}:\n{r.stdout[-2000:]}"
