"""The oracle's pins have teeth: copies of oracle.cpp with one plausible
mistake planted each (a dropped factor, a wrong sign or index, a swapped
operand) are built on the CPU, and the pin suite run against each copy must
fail, while the same suite against an unmodified copy built the same way
passes.  The planted mistakes live only in temporary copies; the oracle
itself is never changed.  (Three pins that take several seconds each are left
out of the runs against the copies; every mistake below is caught without
them.)"""
import concurrent.futures as cf
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.cpp")
PINS = ["tests/test_oracle_topology.py", "tests/test_oracle_dynamics.py", "tests/test_oracle_icm_exact.py",
        "tests/test_oracle_observables.py", "tests/test_oracle_philox.py", "tests/test_oracle_variants.py"]
SKIP = ("not moments_match_exact_enumeration and not chimera_cell_keeps "
        "and not gaussian_disorder_exactly_averaged")

# name -> (text in oracle.cpp, the same text with the mistake)
MUTANTS = {
    "dE without its factor 2": ("int64_t dE = 2 * (int64_t)sp[i] * h;", "int64_t dE = (int64_t)sp[i] * h;"),
    "threshold compared the wrong way": ("    return u < thr;\n", "    return u > thr;\n"),
    "float acceptance without the minus sign":
        ("double p = std::exp(-(beta * std::ldexp((double)dE, -40)));\n  return std::ldexp",
         "double p = std::exp(beta * std::ldexp((double)dE, -40));\n  return std::ldexp"),
    "couplings read in the wrong unit": ("((const float*)p.couplings)[idx], 40)", "((const float*)p.couplings)[idx], 39)"),
    "energy with the wrong sign": ("E -= b.raw * sp[b.i] * sp[b.j];", "E += b.raw * sp[b.i] * sp[b.j];"),
    "cluster flipped in replica a only": ("{ sa[i] = (int8_t)-sa[i]; sb[i] = (int8_t)-sb[i]; ++size; }",
                                          "{ sa[i] = (int8_t)-sa[i]; ++size; }"),
    "seed always the first mask site": ("int idx = (int)(((uint64_t)u * (uint64_t)n) >> 32);", "int idx = 0;"),
    "step 2a at exactly half": ("2 * n > s->N", "2 * n >= s->N"),
    "search follows only higher-numbered neighbours": ("if (mask[j] && label[j] < 0) { label[j] = i;",
                                                       "if (j > v && mask[j] && label[j] < 0) { label[j] = i;"),
    "PT gap with the wrong sign": ("int64_t D = s->energy[y] - s->energy[x];",
                                   "int64_t D = s->energy[x] - s->energy[y];"),
    "PT beta difference reversed": ("double dbeta = s->beta[k] - s->beta[k + 1];",
                                    "double dbeta = s->beta[k + 1] - s->beta[k];"),
    "chimera vertical bond to the wrong site":
        ("if (row + 1 < C) add_bond(s, base + u, 8 * ((row + 1) * C + col) + u, raw);",
         "if (row + 1 < C) add_bond(s, base + u, 8 * ((row + 1) * C + col) + ((u + 1) & 3), raw);"),
    "Philox key schedule swapped": ("k0 += kWeyl0; k1 += kWeyl1;", "k0 += kWeyl1; k1 += kWeyl0;"),
    "hot start from the wrong bit": ("(u >> 31) ? -1 : 1", "((u >> 30) & 1) ? -1 : 1"),
    "link overlap over one end of the bond": ("link += q[e.i] * q[e.j];", "link += q[e.i] * q[e.i];"),
    "time bin off by one": ("while ((t_after >> (bin + 1)) != 0) ++bin;", "while ((t_after >> bin) != 0) ++bin;"),
    "potential cluster sites before step 2a": ("o[3] += std::min(nminus, (int64_t)s->N - nminus);",
                                               "o[3] += nminus;"),
}


def build(text, out_dir):
    cpp = os.path.join(out_dir, "oracle.cpp")
    with open(cpp, "w") as f:
        f.write(text)
    lib = os.path.join(out_dir, "liboracle.so")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-I", os.path.dirname(SRC), cpp,
                           "-o", lib])
    return lib


def run_pins(lib):
    env = dict(os.environ, ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", *PINS, "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                        "-k", SKIP], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


def trial(name, text):
    with tempfile.TemporaryDirectory() as d:
        return name, run_pins(build(text, d))


def test_every_planted_mistake_fails_a_pin():
    with open(SRC) as f:
        src = f.read()
    jobs = {"unmodified": src}
    for name, (old, new) in MUTANTS.items():
        assert src.count(old) == 1, f"{name}: the text to change must occur once in oracle.cpp"
        jobs[name] = src.replace(old, new)
    with cf.ThreadPoolExecutor(min(4, os.cpu_count() or 1)) as ex:
        results = dict(ex.map(lambda kv: trial(*kv), jobs.items()))
    rc, out = results.pop("unmodified")
    assert rc == 0, "the pins must pass on an unmodified copy:\n" + out
    survivors = [name for name, (rc, _) in results.items() if rc == 0]
    assert not survivors, f"planted mistakes no pin catches: {survivors}"
    assert all(rc == 1 for rc, _ in results.values()), {n: r[1] for n, r in results.items() if r[0] != 1}
