"""Load the hand-built events of tests/golden/tiny_events.json."""
import json
import os

import numpy as np

from paper_1906_06242_amd import datagen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "tiny_events.json")


def fnum(x):
    return float(x) if not isinstance(x, str) else float(x.replace("inf", "inf"))


def load():
    with open(GOLDEN) as f:
        g = json.load(f)
    ev = g["events"]
    n = len(ev)

    def coll(key, ncols, names):
        cnt = np.array([len(e[key]) for e in ev], np.int64)
        off = np.zeros(n + 1, np.int64)
        off[1:] = np.cumsum(cnt)
        rows = [r for e in ev for r in e[key]]
        arr = np.array(rows, np.float64).reshape(-1, ncols)
        return datagen.Collection(off, {nm: arr[:, i].astype(np.float32) for i, nm in enumerate(names)})

    jets = coll("jets", 3, ("pt", "eta", "phi"))
    mus = coll("muons", 4, ("pt", "eta", "phi", "iso"))
    w = np.array([e["w"] for e in ev], np.float32)
    ds = datagen.Dataset(n, jets, mus, w)
    q = g["query"]
    query = datagen.Query(mu_pt=q["mu_pt"], mu_abseta=q["mu_abseta"], mu_iso=q["mu_iso"],
                          jet_pt=q["jet_pt"], jet_abseta=q["jet_abseta"], dr=q["dr"],
                          min_mu=q["min_mu"], min_jet=q["min_jet"],
                          edges_ht=datagen.uniform_edges(*q["ht"]),
                          edges_lead=datagen.uniform_edges(*q["lead"]),
                          edges_njet=datagen.uniform_edges(*q["njet"]))
    return g, ds, query


def per_object(g, key, dtype):
    return np.array([fnum(v) for e in g["events"] for v in e[key]], dtype)


def per_event(g, key, dtype):
    return np.array([fnum(e[key]) for e in g["events"]], dtype)


def expected_hist(g, name, nbins):
    s = np.zeros(nbins + 2, np.float64)
    c = np.zeros(nbins + 2, np.uint64)
    for slot, cnt, sw in g["hists"][name]:
        s[slot] = sw
        c[slot] = cnt
    return s, c
