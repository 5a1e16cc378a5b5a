"""Mutation check of the oracle's pins (CPU only).

Each case plants one plausible mistake in a scratch copy of the oracle (a
flipped sign, a swapped index, a dropped term, a wrong rounding or clamp, a
missing conjugate), rebuilds it there, and runs the oracle's pin tests
against the copy: at least one pin must fail.  The unmutated copy must pass,
so a failure is the planted mistake and not the harness.  Every planted text
must occur in the current oracle source, so the list cannot go stale without
this test failing.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
C_SRC = "oracle/afc_oracle.c"
PY_SRC = "oracle/__init__.py"

PIN_FILES = sorted(f for f in os.listdir(os.path.join(ROOT, "tests"))
                   if (f.startswith("test_oracle_") and f.endswith(".py")
                       and f not in ("test_oracle_mutations.py", "test_oracle_sanitizers.py"))
                   or f == "test_workloads.py")

# (name, file, text, replacement, occurrence (0-based) or None if unique)
MUTATIONS = [
    ("dft-sign", C_SRC, "double ang = -2.0 * ORC_PI * (double)r / (double)P;",
     "double ang = 2.0 * ORC_PI * (double)r / (double)P;", None),
    ("tap-order", C_SRC, "double h = (double)taps[t * P + p];",
     "double h = (double)taps[(T - 1 - t) * P + p];", None),
    ("fir-time-index", C_SRC, "int64_t n = (s + t) * P + p;",
     "int64_t n = (s + T - 1 - t) * P + p;", None),
    ("fir-drops-imag", C_SRC, "ai += h * (double)x[2 * (n * row_stride + input) + 1];",
     "ai += h * (double)x[2 * (n * row_stride + input) + 0];", None),
    ("corr-conjugate-side-f64", C_SRC, "im += ai * br - ar * bi;", "im += ar * bi - ai * br;", 0),
    ("corr-conjugate-side-i64", C_SRC, "im += ai * br - ar * bi;", "im += ar * bi - ai * br;", 1),
    ("pair-swap-f64", C_SRC,
     "pair_f64(rows, S, R, pairs[2 * e], pairs[2 * e + 1], out + 2 * e);",
     "pair_f64(rows, S, R, pairs[2 * e + 1], pairs[2 * e], out + 2 * e);", None),
    ("pair-swap-i64", C_SRC,
     "pair_i64(rows, S, R, pairs[2 * e], pairs[2 * e + 1], out + 2 * e);",
     "pair_i64(rows, S, R, pairs[2 * e + 1], pairs[2 * e], out + 2 * e);", None),
    ("pol-layout-f64", C_SRC,
     "V[2 * ((bl * 2 + p) * 2 + q) + 0] = re;\n                    V[2 * ((bl * 2 + p) * 2 + q) + 1] = im;",
     "V[2 * ((bl * 2 + q) * 2 + p) + 0] = re;\n                    V[2 * ((bl * 2 + q) * 2 + p) + 1] = im;", None),
    ("flag-weight-f64", C_SRC, "if (W) W[bl] = flagged ? 0 : (int32_t)S;", "if (W) W[bl] = (int32_t)S;", 0),
    ("flag-weight-i64", C_SRC, "if (W) W[bl] = flagged ? 0 : (int32_t)S;", "if (W) W[bl] = (int32_t)S;", 1),
    ("int32-overflow-missed", C_SRC, "o[1] >= 2147483648LL || o[1] <= -2147483648LL) bad = 1;",
     "o[1] >= 2147483648LL || o[1] <= -2147483648LL) bad = 0;", None),
    ("requant-ties-away", C_SRC, "double r = nearbyint(v);", "double r = round(v);", None),
    ("requant-clamp-128", C_SRC, "if (r < -127.0) r = -127.0;", "if (r < -128.0) r = -128.0;", None),
    ("requant-float32-product", C_SRC, "double v = (double)y[i] * (double)gain;",
     "double v = (double)(y[i] * gain);", None),
    ("cal-missing-conjugate", C_SRC, "Vr[2 * (b * Na + a) + 1] = -vi;", "Vr[2 * (b * Na + a) + 1] = vi;", None),
    ("grad-dropped-term", C_SRC,
     "cr += wba * (r2r * m2r - r2i * m2i);\n                    ci += wba * (r2r * m2i + r2i * m2r);", "", None),
    ("cal-weight-loss-dropped", C_SRC, "L += Wr[a * Na + b] * (rr * rr + ri * ri);", "L += rr * rr + ri * ri;", None),
    ("cal-weight-grad-dropped", C_SRC, "double cr = wab * (rr * mr + ri * mi), ci = wab * (ri * mr - rr * mi);",
     "double cr = (rr * mr + ri * mi), ci = (ri * mr - rr * mi);", None),
    ("cal-weight-pol-index", C_SRC, "w[(ch * nbl + a * (a + 1) / 2 + b) * 2 + pol]",
     "w[(ch * nbl + a * (a + 1) / 2 + b) * 2]", None),
    ("grad-sign", C_SRC, "grad[2 * ((ch * Na + a) * 2 + pol)] = -2.0 * sr;",
     "grad[2 * ((ch * Na + a) * 2 + pol)] = 2.0 * sr;", None),
    ("fine-delay-sign", C_SRC, "const double ang = 2.0 * ORC_PI * (nu_c + fk) * tau;",
     "const double ang = -2.0 * ORC_PI * (nu_c + fk) * tau;", None),
    ("fine-unsigned-offset", C_SRC, "(double)(k < Pf / 2 ? k : k - Pf) * df;", "(double)(k) * df;", None),
    ("validity-short-window", C_SRC, "n < (s + T) * P && ok;", "n < (s + T - 1) * P && ok;", None),
    ("validity-weight-or", C_SRC, "v[a * S_stride + s] && v[b * S_stride + s];",
     "v[a * S_stride + s] || v[b * S_stride + s];", None),
    ("ppf-subband-sorted-inputs", PY_SRC,
     "    inputs = range(R) if inputs is None else list(inputs)\n    out = np.empty((P, S, len(inputs)), np.complex128)",
     "    inputs = range(R) if inputs is None else sorted(inputs)\n    out = np.empty((P, S, len(inputs)), np.complex128)",
     None),
    ("fine-subband-delay-index", PY_SRC, "fine_channelise(x, taps, i, Pf, T, 0, S, tau[i], nu_c, df, w, R).T",
     "fine_channelise(x, taps, i, Pf, T, 0, S, tau[n], nu_c, df, w, R).T", None),
    ("zero-invalid-noop", PY_SRC, "return np.where(keep, z, 0)", "return z", None),
    ("solve-averaging-parity", PY_SRC, "if it % 2 == 0:", "if it % 2 == 1:", None),
    ("solve-weight-numerator", PY_SRC, "num = (Wf * Vf * np.conj(z)).sum(axis=1)", "num = (Vf * np.conj(z)).sum(axis=1)",
     None),
    ("solve-phase-reference", PY_SRC, "g = g * (np.conj(g[0]) / abs(g[0]))", "g = g * (g[0] / abs(g[0]))", None),
    ("clip-rms-includes-flagged", PY_SRC,
     "m = np.where(keep, a2, 0.0).sum(axis=0) / np.maximum(n, 1)", "m = a2.mean(axis=0)", None),
    ("grid-mirror-unconjugated", PY_SRC, "wt[ok] * np.conj(I[ok]))", "wt[ok] * I[ok])", None),
    ("image-no-recentring", PY_SRC, "return (s * F.real) / (norm if norm > 0 else 1.0)",
     "return (F.real) / (norm if norm > 0 else 1.0)", None),
]


def _replace_nth(text, old, new, nth):
    count = text.count(old)
    if nth is None:
        assert count == 1, f"planted text occurs {count} times: {old!r}"
        return text.replace(old, new)
    assert count > nth, f"planted text occurs {count} times, occurrence {nth} asked: {old!r}"
    pos = -1
    for _ in range(nth + 1):
        pos = text.index(old, pos + 1)
    return text[:pos] + new + text[pos + len(old):]


def _scratch_copy(dst):
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(dst, "oracle"),
                    ignore=shutil.ignore_patterns("*.so", "*.so.tmp", "__pycache__"))
    shutil.copytree(os.path.join(ROOT, "workloads"), os.path.join(dst, "workloads"),
                    ignore=shutil.ignore_patterns("__pycache__"))
    os.makedirs(os.path.join(dst, "tests"))
    shutil.copytree(os.path.join(ROOT, "tests", "golden"), os.path.join(dst, "tests", "golden"))
    for f in ["conftest.py", *PIN_FILES]:
        shutil.copy(os.path.join(ROOT, "tests", f), os.path.join(dst, "tests", f))


def _run_pins(dst):
    env = dict(os.environ, OMP_NUM_THREADS="2", PYTHONDONTWRITEBYTECODE="1")
    b = subprocess.run([sys.executable, os.path.join(dst, "oracle", "build.py")], cwd=dst, env=env,
                       capture_output=True, text=True)
    assert b.returncode == 0, b.stdout + b.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        *[os.path.join("tests", f) for f in PIN_FILES]],
                       cwd=dst, env=env, capture_output=True, text=True, timeout=600)
    return r


def _mutant_survives(base, case):
    name, path, old, new, nth = case
    dst = os.path.join(base, name)
    _scratch_copy(dst)
    f = os.path.join(dst, path)
    text = open(f).read()
    open(f, "w").write(_replace_nth(text, old, new, nth))
    r = _run_pins(dst)
    shutil.rmtree(dst, ignore_errors=True)
    # pytest exit code 1: tests ran and at least one failed (not a crash or
    # a collection error, which would be 2..5)
    return None if r.returncode == 1 else f"{name}: pytest exit {r.returncode}\n{r.stdout[-1500:]}"


def test_unmutated_copy_passes(tmp_path):
    _scratch_copy(str(tmp_path))
    r = _run_pins(str(tmp_path))
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]


def test_every_planted_mistake_fails_a_pin(tmp_path):
    names = [m[0] for m in MUTATIONS]
    assert len(set(names)) == len(names)
    workers = max(1, min(8, (os.cpu_count() or 2) // 2))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        survivors = [s for s in ex.map(lambda m: _mutant_survives(str(tmp_path), m), MUTATIONS) if s]
    assert not survivors, "planted mistakes that no pin caught:\n" + "\n".join(survivors)
