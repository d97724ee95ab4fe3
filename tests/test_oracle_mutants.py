"""The oracle's pins have teeth: each planted mistake must fail a pin.

Every mutant is a copy of oracle/hepkref.c with one plausible slip (dropped
wrap, wrong boundary, wrong index base, summation order, ...), compiled with
gcc into a temporary directory and run against tests/test_oracle_pins.py in
a subprocess.  CPU only; nothing here touches the GPU library.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hepkref.c")

MUTANTS = [
    ("no phi wrap", "if (dphi > REF_PI)", "if (0)"),
    ("lower wrap dropped", "else if (dphi < -REF_PI)", "else if (0)"),
    ("strict cone", "!(best <= thr2)", "!(best < thr2)"),
    ("double-precision sum", "float acc = 0.0f;", "double acc = 0.0;"),
    ("max tie to last", "int better = want_max ? (v > best) : (v < best);",
     "int better = want_max ? (v >= best) : (v <= best);"),
    ("bins closed on the right", "if (v < edges[k + 1])", "if (v <= edges[k + 1])"),
    ("dR cross term", "deta * deta + dphi * dphi", "deta * deta + deta * dphi"),
    ("global instead of local index", "bi = (int32_t)(b - off_b[e]);", "bi = (int32_t)(b);"),
    ("bin slot off by one", "b = k + 1;", "b = k;"),
    ("cuts ORed", "pass = pass && ok;", "pass = pass || ok;"),
    ("isolation cut dropped", "if (ds->muons.extra) mc[nmc++]", "if (0) mc[nmc++]"),
    ("half exponent bias", "(int)ex - 25", "(int)ex - 24"),
    ("eta difference sign", "float deta = ea - load_f(eta_b, dtype, b);",
     "float deta = ea + load_f(eta_b, dtype, b);"),
    ("scale not applied", "ptv[j] = load_f(ds->jets.pt, dt, j) * s;", "ptv[j] = load_f(ds->jets.pt, dt, j);"),
    ("electron cleaning loses muon cleaning",
     "hepkref_match_dr(ds->jets.off, ds->jets.eta, ds->jets.phi, clean,",
     "hepkref_match_dr(ds->jets.off, ds->jets.eta, ds->jets.phi, NULL,"),
    ("lead on unscaled pt", "hepkref_reduce(HEPKREF_MAX, ds->jets.off, N, ptv, HEPKREF_F32",
     "hepkref_reduce(HEPKREF_MAX, ds->jets.off, N, ds->jets.pt, dt"),
    ("underflow into first bin", "b = 0;\n        } else {", "b = 1;\n        } else {"),
    ("weights ignored", "sumw[b] += (double)(w ? w[i] : 1.0f);", "sumw[b] += 1.0;"),
    ("prefix offsets shifted", "if (offsets_out) offsets_out[e + 1] = running;",
     "if (offsets_out) offsets_out[e] = running;"),
    ("b-tag read from pt", "hepkref_cut bc = mkcut(ds->jets.extra", "hepkref_cut bc = mkcut(ds->jets.pt"),
    ("b-jet requirement ignored", "ev[nev++] = mkicut(n_b, HEPKREF_GE, q->min_b);", "(void)0;"),
    ("H_T over unselected jets", "hepkref_reduce(HEPKREF_SUM, ds->jets.off, N, ptv, HEPKREF_F32, jsel",
     "hepkref_reduce(HEPKREF_SUM, ds->jets.off, N, ptv, HEPKREF_F32, NULL"),
    ("interpolation slope inverted", "/ (bin_centre(edges, i + 1) - m_i);", "/ (m_i - bin_centre(edges, i + 1));"),
    ("interpolation clamps to the underflow slot", "if (v <= bin_centre(edges, 1)) return c[1];",
     "if (v <= bin_centre(edges, 1)) return c[0];"),
    ("lookup slot excludes its lower edge", "if (edges[k] <= v) s++;", "if (edges[k] < v) s++;"),
    ("JES row from signed eta", "float ae = fabsf(load_f(eta, dtype, i));", "float ae = load_f(eta, dtype, i);"),
    ("product starts at zero", "float prod = 1.0f;", "float prod = 0.0f;"),
    ("sumw2 adds the weight", "sumw2[b] += wi * wi;", "sumw2[b] += wi;"),
    ("pileup weight ignored", "for (int64_t e = 0; e < N; e++) wev[e] = wev[e] * evf[e];", "(void)0;"),
    ("scale factors of unselected muons",
     "hepkref_reduce(HEPKREF_PROD, ds->muons.off, N, mu_sf, HEPKREF_F32, msel,",
     "hepkref_reduce(HEPKREF_PROD, ds->muons.off, N, mu_sf, HEPKREF_F32, NULL,"),
    ("lookup JES shift dropped", "(1.0f + s * delta[j])", "(1.0f + delta[j])"),
    ("n-th object counts unselected ones", "        if (obj_mask && !obj_mask[i]) continue;\n        if (seen == n) return i;",
     "        if (seen == n) return i;"),
    ("n-th object as a global index", "out_index[e] = (i >= 0) ? (int32_t)(i - offsets[e]) : -1;",
     "out_index[e] = (i >= 0) ? (int32_t)i : -1;"),
    ("mask set ignores the value", "((uint8_t *)content)[i] = (value != 0.0f) ? 1 : 0;",
     "((uint8_t *)content)[i] = 1;"),
    ("opposite sign as different charge", "return (a > 0 && b < 0) || (a < 0 && b > 0);", "return a != b;"),
    ("pT order ascending", "if (!ni && pi != pj) return pi > pj;", "if (!ni && pi != pj) return pi < pj;"),
    ("every opposite pair kept", "                    found = 1;", "                    found = 0;"),
    ("compaction ignores the mask",
     "            if (obj_mask && !obj_mask[i]) continue;\n            memcpy(", "            memcpy("),
    ("triplet ties to the last", "if (d < best_d) {", "if (d <= best_d) {"),
    ("triplet energy summed in another order", "float se = (en[i] + en[j]) + en[k];",
     "float se = en[i] + (en[j] + en[k]);"),
    ("p4 py from cos", "y = p * sin(f)", "y = p * cos(f)"),
    ("event mask ignored by count",
     "if (take_event)\n                for (int64_t i = i0; i < i1; i++)\n                    if (!obj_mask",
     "if (1)\n                for (int64_t i = i0; i < i1; i++)\n                    if (!obj_mask"),
]


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site vanished: {name}"
    mut = os.path.join(tmp_path, "hepkref.c")
    with open(mut, "w") as f:
        f.write(src.replace(old, new, 1))
    with open(os.path.join(tmp_path, "hepkref.h"), "w") as f:
        f.write(open(os.path.join(ROOT, "oracle", "hepkref.h")).read())
    so = os.path.join(tmp_path, "libmut.so")
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                           "-o", so, mut, "-lm"], stderr=subprocess.DEVNULL)
    env = dict(os.environ, HEPKREF_LIB=so)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_pins_positional.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode != 0, f"mutant '{name}' passed every pin:\n{r.stdout[-500:]}"
