"""The analysis pass as a chain of single-purpose kernel calls.

This is how Sec. III proposes to steer an analysis from high-level code --
one kernel call per step, masks and per-event arrays passed from call to call
through device memory -- and how Sec. IV's benchmark ran (hundreds of calls
per pass).  Each step is one call into libhepk; intermediates round-trip HBM.
It computes the same histograms as the fused hepk_pipeline and serves as its
per-kernel baseline.  Only the nominal jet-energy scale (1.0) is supported:
scaled pt would need one more elementwise kernel per variation.
"""
from __future__ import annotations

from typing import List, Tuple

from . import hepk as H


def run(dd: "H.DeviceDataset", q, hists=None, stream=None) -> List[Tuple]:
    """One pass for query q over device dataset dd.

    hists: optional [(sumw, counts)] * 3 device tensors to accumulate into.
    Returns the three (sumw, counts) pairs (H_T, leading pt, nJet).
    """
    import torch
    if q.n_scale != 1 or float(q.scales[0]) != 1.0:
        raise ValueError("the per-kernel pipeline runs the nominal scale only")
    t = dd.t
    n = dd.n_events
    mm = t("muons.pt").numel()
    mj = t("jets.pt").numel()
    if hists is None:
        hists = []
        for e in q.edges():
            nb = len(e) - 1
            hists.append((torch.zeros(nb + 2, dtype=torch.float64, device="cuda"),
                          torch.zeros(nb + 2, dtype=torch.int64, device="cuda")))
    edges = [torch.from_numpy(e.astype("float32")).to("cuda") for e in q.edges()]

    mcuts = [(t("muons.pt"), H.GT, q.mu_pt), (t("muons.eta"), H.ABS_LT, q.mu_abseta)]
    if t("muons.iso") is not None:
        mcuts.append((t("muons.iso"), H.LT, q.mu_iso))
    msel = H.select(mcuts, mm, stream=stream)
    nmu = H.reduce(H.COUNT, t("muons.offsets"), obj_mask=msel, stream=stream)
    _, _, clean = H.match_dr(t("jets.offsets"), t("jets.eta"), t("jets.phi"),
                             t("muons.offsets"), t("muons.eta"), t("muons.phi"), q.dr,
                             mask_b=msel, want=("clean",), stream=stream)
    if dd.has_electrons:
        me = t("electrons.pt").numel()
        esel = H.select([(t("electrons.pt"), H.GT, q.el_pt),
                         (t("electrons.eta"), H.ABS_LT, q.el_abseta)], me, stream=stream)
        _, _, clean = H.match_dr(t("jets.offsets"), t("jets.eta"), t("jets.phi"),
                                 t("electrons.offsets"), t("electrons.eta"), t("electrons.phi"),
                                 q.dr, mask_a=clean, mask_b=esel, want=("clean",), stream=stream)
    jsel = H.select([(t("jets.pt"), H.GT, q.jet_pt), (t("jets.eta"), H.ABS_LT, q.jet_abseta)],
                    mj, mask_in=clean, stream=stream)
    njet = H.reduce(H.COUNT, t("jets.offsets"), obj_mask=jsel, stream=stream)
    ht = H.reduce(H.SUM, t("jets.offsets"), t("jets.pt"), obj_mask=jsel, stream=stream)
    lead = H.reduce(H.MAX, t("jets.offsets"), t("jets.pt"), obj_mask=jsel, stream=stream)
    ecuts = [(nmu, H.GE, q.min_mu), (njet, H.GE, q.min_jet)]
    if t("jets.btag") is not None:
        bsel = H.select([(t("jets.btag"), H.GT, q.btag)], mj, mask_in=jsel, stream=stream)
        nb = H.reduce(H.COUNT, t("jets.offsets"), obj_mask=bsel, stream=stream)
        ecuts.append((nb, H.GE, q.min_b))
    passed = H.select(ecuts, n, stream=stream)
    w = t("weight")
    for x, e, (s, c) in zip((ht, lead, njet), edges, hists):
        H.hist_fill(x, e, s, c, w=w, evt_mask=passed, stream=stream)
    return hists
