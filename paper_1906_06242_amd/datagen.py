"""Seeded synthetic collider events stored as jagged columns.

Events follow the jagged layout of Sec. II: per collection an int64
``offsets`` array of N+1 entries and one contiguous content array of M
entries per feature, ``offsets[e]:offsets[e+1]`` being the objects of event
e.  The CMS Open Data of Sec. IV is not available, so these draws stand in
for it with the shapes of the paper's workload (jets, muons and, in the
extended schema, electrons; pt/eta/phi/mass kinematics; a per-event weight).

This module holds inputs only -- event content, histogram bin edges,
jet-energy-scale factors and query parameters -- and none of the analysis
arithmetic.  Both the HIP library and the CPU oracle consume what it makes.

Draws are made in float64 with ``numpy.random.default_rng`` and cast once
to the storage dtype.  Generation is split into chunks of ``CHUNK`` events,
chunk c of seed s drawn from ``default_rng([s, c])``, so a dataset is
defined independently of how many chunks are generated at once and large
datasets can be generated in parallel or streamed.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field
from typing import Dict, Iterator, List, Optional

import numpy as np

CHUNK = 1 << 20  # events per independently seeded chunk

# Column names of each collection, in draw order.
JET_COLS = ("pt", "eta", "phi", "mass")
MU_COLS = ("pt", "eta", "phi", "mass", "iso")
EL_COLS = ("pt", "eta", "phi", "mass")


@dataclass
class Collection:
    """One jagged collection: offsets (int64, N+1) and named content columns."""
    offsets: np.ndarray
    cols: Dict[str, np.ndarray] = field(default_factory=dict)

    @property
    def n_objects(self) -> int:
        return int(self.offsets[-1])


@dataclass
class Dataset:
    """Events of one sample: jets, muons, optional electrons, event weights."""
    n_events: int
    jets: Collection
    muons: Collection
    weight: np.ndarray                     # float32[N]
    electrons: Optional[Collection] = None
    content_dtype: str = "f32"             # "f32" or "f16"
    seed: int = 0
    npu: Optional[np.ndarray] = None       # float32[N] pileup per event (with_pileup)

    def collections(self):
        out = [("jets", self.jets), ("muons", self.muons)]
        if self.electrons is not None:
            out.append(("electrons", self.electrons))
        return out

    def nbytes_read(self) -> int:
        """Bytes of the columns the analysis reads (mass columns excluded)."""
        esz = 2 if self.content_dtype == "f16" else 4
        b = 8 * (self.n_events + 1) * 2 + 4 * self.n_events
        b += esz * self.jets.n_objects * (4 if "btag" in self.jets.cols else 3)
        b += esz * self.muons.n_objects * 4
        if self.electrons is not None:
            b += 8 * (self.n_events + 1) + esz * self.electrons.n_objects * 3
        return b

    def nbytes_read_lookup(self) -> int:
        """Bytes read by a pass that also takes the pileup column."""
        return self.nbytes_read() + (4 * self.n_events if self.npu is not None else 0)

    def nbytes_stored(self) -> int:
        b = self.weight.nbytes
        for _, c in self.collections():
            b += c.offsets.nbytes + sum(a.nbytes for a in c.cols.values())
        return b


def _offsets(counts: np.ndarray) -> np.ndarray:
    off = np.zeros(len(counts) + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    return off


def _draw_chunk(seed: int, c: int, n: int, extended: bool):
    """Draw chunk c (n events) of the dataset with this seed.

    Returns (counts dict, content dict of float64 arrays, weight float64).
    Order of draws: multiplicities, weight, jet columns, muon columns,
    then (extended) electron columns and the jet b-tag score.
    """
    rng = np.random.default_rng([seed, c])
    nj = np.minimum(rng.poisson(5.0, n), 20)
    nm = np.minimum(rng.poisson(1.5, n), 8)
    ne = np.minimum(rng.poisson(0.8, n), 8) if extended else None
    w = rng.normal(1.0, 0.1, n)
    mj, mm = int(nj.sum()), int(nm.sum())
    jets = {
        "pt": 20.0 + rng.exponential(30.0, mj),
        "eta": np.clip(rng.normal(0.0, 1.5, mj), -4.7, 4.7),
        "phi": rng.uniform(-math.pi, math.pi, mj),
        "mass": rng.uniform(0.0, 20.0, mj),
    }
    mus = {
        "pt": 20.0 + rng.exponential(30.0, mm),
        "eta": np.clip(rng.normal(0.0, 1.5, mm), -4.7, 4.7),
        "phi": rng.uniform(-math.pi, math.pi, mm),
        "mass": rng.uniform(0.0, 20.0, mm),
        "iso": rng.exponential(0.1, mm),
    }
    els = None
    if extended:
        me = int(ne.sum())
        els = {
            "pt": 20.0 + rng.exponential(30.0, me),
            "eta": np.clip(rng.normal(0.0, 1.5, me), -4.7, 4.7),
            "phi": rng.uniform(-math.pi, math.pi, me),
            "mass": rng.uniform(0.0, 20.0, me),
        }
        jets["btag"] = rng.beta(0.5, 2.0, mj)
    counts = {"jets": nj, "muons": nm}
    if extended:
        counts["electrons"] = ne
    cont = {"jets": jets, "muons": mus}
    if extended:
        cont["electrons"] = els
    return counts, cont, w


def _chunk_sizes(n_events: int):
    n_full, rem = divmod(n_events, CHUNK)
    return [CHUNK] * n_full + ([rem] if rem else [])


def iter_chunks(seed: int, n_events: int, extended: bool = False,
                content_dtype: str = "f32", start_chunk: int = 0
                ) -> Iterator[Dataset]:
    """Yield the dataset chunk by chunk, each a Dataset with local offsets."""
    cdt = np.float16 if content_dtype == "f16" else np.float32
    for c, n in enumerate(_chunk_sizes(n_events)):
        if c < start_chunk:
            continue
        counts, cont, w = _draw_chunk(seed, c, n, extended)
        colls = {}
        for name, cnt in counts.items():
            colls[name] = Collection(_offsets(cnt),
                                     {k: v.astype(cdt) for k, v in cont[name].items()})
        yield Dataset(n, colls["jets"], colls["muons"], w.astype(np.float32),
                      colls.get("electrons"), content_dtype, seed)


def concat(parts: List[Dataset]) -> Dataset:
    """Concatenate chunk datasets into one (offsets rebased)."""
    def cat_coll(cs: List[Collection]) -> Collection:
        offs, base = [np.zeros(1, np.int64)], 0
        for c in cs:
            offs.append(c.offsets[1:] + base)
            base += c.n_objects
        cols = {k: np.concatenate([c.cols[k] for c in cs]) for k in cs[0].cols}
        return Collection(np.concatenate(offs), cols)
    p0 = parts[0]
    return Dataset(sum(p.n_events for p in parts),
                   cat_coll([p.jets for p in parts]),
                   cat_coll([p.muons for p in parts]),
                   np.concatenate([p.weight for p in parts]),
                   cat_coll([p.electrons for p in parts]) if p0.electrons is not None else None,
                   p0.content_dtype, p0.seed)


def _chunk_job(args):
    seed, c, n, extended, content_dtype = args
    return next(iter_chunks(seed, (c + 1) * CHUNK if n == CHUNK else c * CHUNK + n,
                            extended, content_dtype, start_chunk=c))


def make_dataset(seed: int, n_events: int, extended: bool = False,
                 content_dtype: str = "f32", jobs: int = 0) -> Dataset:
    """The whole dataset in host memory.

    jobs > 1 draws the chunks in that many processes (same result: every
    chunk has its own seed).  jobs = 0 picks min(8, cpus) for large datasets,
    or HEPK_GEN_JOBS if set (1 for processes that must not fork, e.g. under a
    profiler that has already opened the GPU).
    """
    if n_events == 0:
        z = np.zeros(1, np.int64)
        cdt = np.float16 if content_dtype == "f16" else np.float32
        mk = lambda cols: Collection(z.copy(), {k: np.zeros(0, cdt) for k in cols})
        jc = JET_COLS + (("btag",) if extended else ())
        return Dataset(0, mk(jc), mk(MU_COLS), np.zeros(0, np.float32),
                       mk(EL_COLS) if extended else None, content_dtype, seed)
    sizes = _chunk_sizes(n_events)
    if jobs == 0:
        jobs = int(os.environ.get("HEPK_GEN_JOBS", "0")) or (min(8, os.cpu_count() or 1) if len(sizes) > 2 else 1)
    if jobs <= 1 or len(sizes) == 1:
        return concat(list(iter_chunks(seed, n_events, extended, content_dtype)))
    import multiprocessing as mp
    with mp.get_context("fork").Pool(min(jobs, len(sizes))) as pool:
        parts = pool.map(_chunk_job, [(seed, c, n, extended, content_dtype)
                                      for c, n in enumerate(sizes)])
    return concat(parts)


# ---------------------------------------------------------------------------
# analysis inputs
# ---------------------------------------------------------------------------

def uniform_edges(nbins: int, lo: float, hi: float) -> np.ndarray:
    """nbins+1 float32 edges lo + (hi-lo)*i/nbins, computed in float64."""
    i = np.arange(nbins + 1, dtype=np.float64)
    return (lo + (hi - lo) * i / nbins).astype(np.float32)


def jes_scales(n_steps: int = 10, step: float = 0.01) -> np.ndarray:
    """Jet-energy-scale factors 1+k*step (k=1..n) then 1-k*step, float32."""
    up = [1.0 + k * step for k in range(1, n_steps + 1)]
    dn = [1.0 - k * step for k in range(1, n_steps + 1)]
    return np.array(up + dn, dtype=np.float64).astype(np.float32)


def with_pileup(ds: Dataset, seed: int, mean: float = 20.0) -> Dataset:
    """A copy of ds with a pileup column: the number of simultaneous
    interactions per event, Poisson(mean), stored as float32 (drawn from its
    own stream, default_rng([seed, 0x50550])) -- the per-event variable of
    pileup reweighting."""
    rng = np.random.default_rng([seed, 0x50550])
    npu = rng.poisson(mean, ds.n_events).astype(np.float32)
    return Dataset(ds.n_events, ds.jets, ds.muons, ds.weight, ds.electrons, ds.content_dtype, ds.seed, npu)


def muon_charges(ds: Dataset, seed: int) -> np.ndarray:
    """A charge per muon, +1 or -1 with equal probability, int32 (drawn from
    its own stream, default_rng([seed, 0xC4A6])) -- the column the
    opposite-sign selection reads."""
    rng = np.random.default_rng([seed, 0xC4A6])
    return np.where(rng.uniform(size=ds.muons.n_objects) < 0.5, 1, -1).astype(np.int32)


def pileup_table(data_mean: float = 22.0, sim_mean: float = 20.0, nbins: int = 80):
    """Synthetic pileup-reweighting table (edges, contents): in unit bins of
    the pileup count 0..nbins, the ratio of Poisson(data_mean) to
    Poisson(sim_mean) probabilities; 1 in the under- and overflow slots."""
    k = np.arange(nbins, dtype=np.float64)
    lg = np.array([math.lgamma(x + 1.0) for x in k])
    ratio = np.exp(k * math.log(data_mean) - data_mean - lg - (k * math.log(sim_mean) - sim_mean - lg))
    contents = np.concatenate([[1.0], ratio, [1.0]]).astype(np.float32)
    return uniform_edges(nbins, 0.0, float(nbins)), contents


def muon_sf_table():
    """Synthetic muon efficiency scale factors (edges, contents) in muon pt:
    rising from 0.95 towards 0.99; under/overflow take the nearest bin's
    value."""
    edges = np.array([20, 25, 30, 40, 50, 60, 80, 120, 200, 500], np.float64)
    centres = 0.5 * (edges[:-1] + edges[1:])
    sf = 0.95 + 0.04 * (1.0 - np.exp(-(centres - 20.0) / 30.0))
    contents = np.concatenate([[sf[0]], sf, [sf[-1]]]).astype(np.float32)
    return edges.astype(np.float32), contents


def jes_table():
    """Synthetic in-situ jet-energy-scale uncertainty (eta_edges, pt_edges,
    delta[n_eta, n_pt]): rows of |eta| bins, values at log-spaced pt bin
    centres, larger at low pt and forward |eta|."""
    eta_edges = np.array([0.0, 0.5, 1.0, 1.5, 2.0, 2.5, 3.0, 4.7], np.float64)
    pt_edges = np.geomspace(20.0, 1000.0, 25)
    cpt = np.sqrt(pt_edges[:-1] * pt_edges[1:])
    rows = np.arange(len(eta_edges) - 1, dtype=np.float64)[:, None]
    delta = 0.015 + 0.06 * np.exp(-cpt[None, :] / 60.0) + 0.004 * rows
    return eta_edges.astype(np.float32), pt_edges.astype(np.float32), delta.astype(np.float32)


def jes_lookup_shifts(n_steps: int = 10, step: float = 0.5) -> np.ndarray:
    """Shifts k of the lookup jet-energy scale pt * (1 + k * delta): +k*step
    then -k*step for k = 1..n_steps, float32."""
    up = [k * step for k in range(1, n_steps + 1)]
    return np.array(up + [-x for x in up], dtype=np.float64).astype(np.float32)


@dataclass
class Query:
    """Cuts, event requirements and binnings of one analysis pass.

    Object cuts: muon pt > mu_pt, |eta| < mu_abseta, iso < mu_iso; electron
    pt > el_pt, |eta| < el_abseta; jet pt*scale > jet_pt, |eta| < jet_abseta,
    no selected lepton within dr; b-tagged jet: selected and btag > btag.
    Event: nMu >= min_mu, nJet >= min_jet, nB >= min_b.
    Histograms (HT, leading-jet pt, nJet) per jet-energy scale.
    """
    mu_pt: float = 20.0
    mu_abseta: float = 2.4
    mu_iso: float = 0.15
    el_pt: float = 20.0
    el_abseta: float = 2.5
    jet_pt: float = 30.0
    jet_abseta: float = 2.5
    dr: float = 0.4
    btag: float = 0.5
    min_mu: int = 1
    min_jet: int = 4
    min_b: int = 0
    scales: np.ndarray = field(default_factory=lambda: np.ones(1, np.float32))
    edges_ht: np.ndarray = field(default_factory=lambda: uniform_edges(100, 0.0, 2000.0))
    edges_lead: np.ndarray = field(default_factory=lambda: uniform_edges(100, 0.0, 1000.0))
    edges_njet: np.ndarray = field(default_factory=lambda: uniform_edges(21, 0.0, 21.0))
    arrival: float = 0.0                   # seconds (serving stream only)
    # lookup corrections (None: absent): event weight w * pu(npu) * product of
    # sf(pt) over selected muons; jet energy scale pt * (1 + s * delta(pt, |eta|))
    # with the scales read as shifts s (jes = (eta_edges, pt_edges, delta))
    pu: Optional[tuple] = None             # (edges, contents[nbins+2])
    sf: Optional[tuple] = None             # (edges, contents[nbins+2])
    jes: Optional[tuple] = None

    def edges(self):
        return (self.edges_ht, self.edges_lead, self.edges_njet)

    @property
    def n_scale(self) -> int:
        return int(len(self.scales))


def extended_query() -> Query:
    """Extended schema: b-tag requirement and 20 jet-energy-scale variations."""
    return Query(min_b=1, scales=jes_scales())


def lookup_query(min_b: int = 1) -> Query:
    """Lookup corrections: pileup and muon scale-factor event weights and 20
    jet-energy-scale variations from the interpolated uncertainty table."""
    return Query(min_b=min_b, scales=jes_lookup_shifts(), pu=pileup_table(), sf=muon_sf_table(),
                 jes=jes_table())


def batch_sizes(seed: int = 0, n: int = 64, lo: float = 1e4, hi: float = 5e6) -> np.ndarray:
    """Event counts log-uniform in [lo, hi] for a batch of uneven datasets."""
    rng = np.random.default_rng(seed)
    return np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), n))).astype(np.int64)


def draw_queries(seed: int, n: int, qps: float = 50.0) -> List[Query]:
    """Poisson stream of queries with random cut thresholds and binnings."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / qps, n)
    t = np.cumsum(gaps)
    mu_pt = rng.uniform(15.0, 40.0, n).astype(np.float32)
    jet_pt = rng.uniform(25.0, 60.0, n).astype(np.float32)
    min_jet = rng.integers(2, 7, n)
    nb_ht = rng.integers(50, 201, n)
    nb_lead = rng.integers(50, 201, n)
    out = []
    for i in range(n):
        out.append(Query(mu_pt=float(mu_pt[i]), jet_pt=float(jet_pt[i]),
                         min_jet=int(min_jet[i]),
                         edges_ht=uniform_edges(int(nb_ht[i]), 0.0, 2000.0),
                         edges_lead=uniform_edges(int(nb_lead[i]), 0.0, 1000.0),
                         arrival=float(t[i])))
    return out


# ---------------------------------------------------------------------------
# on-device generation for the large workloads
# ---------------------------------------------------------------------------

DEVICE_CHUNK = 1 << 22  # events per independently seeded device chunk


def make_dataset_device(seed: int, n_events: int, extended: bool = False,
                        content_dtype: str = "f32", device: str = "cuda"):
    """The same distributions drawn on the GPU (torch Philox streams).

    Chunk c of seed s uses generator seed s * 1_000_003 + c; draws are float64,
    cast once to the storage dtype.  Returns a dict of device tensors with the
    keys of paper_1906_06242_amd.hepk.DeviceDataset ("jets.offsets",
    "jets.pt", ..., "weight") plus "n_events".  A different random stream
    from make_dataset (which draws on the host), so the two generators give
    different events with the same distributions.
    """
    import torch
    dev = device
    cdt = torch.float16 if content_dtype == "f16" else torch.float32
    parts = {}
    bases = {"jets": 0, "muons": 0, "electrons": 0}
    names = {"jets": ["pt", "eta", "phi", "mass"] + (["btag"] if extended else []),
             "muons": ["pt", "eta", "phi", "mass", "iso"],
             "electrons": ["pt", "eta", "phi", "mass"]}
    colls = ["jets", "muons"] + (["electrons"] if extended else [])
    rates = {"jets": (5.0, 20), "muons": (1.5, 8), "electrons": (0.8, 8)}
    for c in range((n_events + DEVICE_CHUNK - 1) // DEVICE_CHUNK):
        n = min(DEVICE_CHUNK, n_events - c * DEVICE_CHUNK)
        g = torch.Generator(device=dev)
        g.manual_seed(seed * 1_000_003 + c)
        counts = {}
        for name in colls:
            lam, cap = rates[name]
            k = torch.poisson(torch.full((n,), lam, dtype=torch.float64, device=dev), generator=g)
            counts[name] = torch.clamp(k, max=cap).to(torch.int64)
        w = torch.empty(n, dtype=torch.float64, device=dev).normal_(1.0, 0.1, generator=g)
        parts.setdefault("weight", []).append(w.to(torch.float32))
        for name in colls:
            m = int(counts[name].sum())
            off = torch.cumsum(counts[name], 0) + bases[name]
            parts.setdefault(f"{name}.offsets", []).append(off)
            bases[name] += m
            pt = 20.0 + torch.empty(m, dtype=torch.float64, device=dev).exponential_(1.0 / 30.0, generator=g)
            eta = torch.clamp(torch.empty(m, dtype=torch.float64, device=dev).normal_(0.0, 1.5, generator=g), -4.7, 4.7)
            phi = torch.empty(m, dtype=torch.float64, device=dev).uniform_(-math.pi, math.pi, generator=g)
            mass = torch.empty(m, dtype=torch.float64, device=dev).uniform_(0.0, 20.0, generator=g)
            cols = {"pt": pt, "eta": eta, "phi": phi, "mass": mass}
            if name == "muons":
                cols["iso"] = torch.empty(m, dtype=torch.float64, device=dev).exponential_(1.0 / 0.1, generator=g)
            if name == "jets" and extended:
                a = torch._standard_gamma(torch.full((m,), 0.5, dtype=torch.float64, device=dev), generator=g)
                b = torch._standard_gamma(torch.full((m,), 2.0, dtype=torch.float64, device=dev), generator=g)
                cols["btag"] = a / (a + b)
            for k in names[name]:
                parts.setdefault(f"{name}.{k}", []).append(cols[k].to(cdt))
    out = {"n_events": n_events, "content_dtype": content_dtype}
    for key, lst in parts.items():
        if key.endswith(".offsets"):
            out[key] = torch.cat([torch.zeros(1, dtype=torch.int64, device=dev)] + lst)
        else:
            out[key] = torch.cat(lst) if lst else torch.zeros(0, device=dev)
    if n_events == 0:
        for name in colls:
            out[f"{name}.offsets"] = torch.zeros(1, dtype=torch.int64, device=dev)
    return out


def host_slice(dev_ds: dict, e0: int, e1: int) -> Dataset:
    """Host copy of events [e0, e1) of an on-device dataset (offsets rebased)."""
    colls = [c for c in ("jets", "muons", "electrons") if f"{c}.offsets" in dev_ds]
    built = {}
    for name in colls:
        off = dev_ds[f"{name}.offsets"][e0:e1 + 1].cpu().numpy()
        a, b = int(off[0]), int(off[-1])
        cols = {}
        for key, t in dev_ds.items():
            if isinstance(key, str) and key.startswith(name + ".") and not key.endswith(".offsets"):
                cols[key.split(".", 1)[1]] = t[a:b].cpu().numpy()
        built[name] = Collection(off - a, cols)
    w = dev_ds["weight"][e0:e1].cpu().numpy()
    npu = dev_ds["npu"][e0:e1].cpu().numpy() if "npu" in dev_ds else None
    return Dataset(e1 - e0, built["jets"], built["muons"], w, built.get("electrons"),
                   dev_ds.get("content_dtype", "f32"), npu=npu)


def with_pileup_device(dev_ds: dict, seed: int, mean: float = 20.0) -> dict:
    """The on-device dataset with a pileup column, Poisson(mean) as float32,
    drawn on the GPU (generator seed seed * 1_000_003 + 0x50550)."""
    import torch
    n = int(dev_ds["n_events"])
    dev = dev_ds["weight"].device
    g = torch.Generator(device=dev)
    g.manual_seed(seed * 1_000_003 + 0x50550)
    lam = torch.full((max(n, 1),), mean, dtype=torch.float64, device=dev)
    out = dict(dev_ds)
    out["npu"] = torch.poisson(lam, generator=g).to(torch.float32)[:max(n, 1)]
    return out
