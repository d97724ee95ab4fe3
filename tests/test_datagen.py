"""The seeded input generators: shapes, caps, distributions, determinism."""
import numpy as np

from paper_1906_06242_amd import datagen


def test_host_generator_shapes_caps_and_moments():
    ds = datagen.make_dataset(0, 200000)
    nj = np.diff(ds.jets.offsets)
    nm = np.diff(ds.muons.offsets)
    assert nj.max() <= 20 and nm.max() <= 8 and nj.min() >= 0
    assert abs(nj.mean() - 5.0) < 0.02 and abs(nm.mean() - 1.5) < 0.01
    pt = ds.jets.cols["pt"].astype(np.float64)
    assert pt.min() >= 20.0 and abs(pt.mean() - 50.0) < 0.2
    eta = ds.jets.cols["eta"]
    assert np.abs(eta).max() <= np.float32(4.7) and abs(eta.std() - 1.5) < 0.01
    assert abs(ds.muons.cols["iso"].mean() - 0.1) < 0.002
    assert abs(ds.weight.mean() - 1.0) < 0.001 and ds.weight.dtype == np.float32
    assert ds.jets.cols["pt"].dtype == np.float32 and ds.jets.offsets.dtype == np.int64


def test_host_generator_is_deterministic_and_chunk_independent():
    a = datagen.make_dataset(3, datagen.CHUNK + 10, jobs=1)
    b = datagen.make_dataset(3, datagen.CHUNK + 10, jobs=2)
    assert np.array_equal(a.jets.offsets, b.jets.offsets)
    assert np.array_equal(a.muons.cols["phi"], b.muons.cols["phi"])
    c = datagen.make_dataset(3, 1000)
    assert np.array_equal(a.jets.offsets[:1001], c.jets.offsets)


def test_extended_schema_f16():
    ds = datagen.make_dataset(1, 50000, extended=True, content_dtype="f16")
    assert ds.electrons is not None and ds.jets.cols["btag"].dtype == np.float16
    bt = ds.jets.cols["btag"].astype(np.float64)
    assert 0.0 <= bt.min() and bt.max() <= 1.0 and abs(bt.mean() - 0.2) < 0.005
    assert abs(np.diff(ds.electrons.offsets).mean() - 0.8) < 0.02


def test_device_generator_on_cpu_and_host_slice():
    t = datagen.make_dataset_device(5, 30000, extended=True, device="cpu")
    nj = np.diff(t["jets.offsets"].numpy())
    assert nj.max() <= 20 and abs(nj.mean() - 5.0) < 0.1
    assert t["jets.pt"].numel() == int(t["jets.offsets"][-1])
    assert t["muons.iso"].numel() == int(t["muons.offsets"][-1])
    assert abs(float(t["muons.iso"].double().mean()) - 0.1) < 0.01
    s = datagen.host_slice(t, 1000, 1500)
    assert s.n_events == 500 and s.jets.offsets[0] == 0
    assert s.jets.n_objects == int(t["jets.offsets"][1500] - t["jets.offsets"][1000])
    t2 = datagen.make_dataset_device(5, 30000, extended=True, device="cpu")
    assert all(np.array_equal(t[k].numpy(), t2[k].numpy()) for k in t if hasattr(t[k], "numpy"))


def test_edges_scales_batches_queries():
    e = datagen.uniform_edges(100, 0.0, 2000.0)
    assert e.dtype == np.float32 and e[0] == 0 and e[-1] == 2000 and np.all(np.diff(e) > 0)
    s = datagen.jes_scales()
    assert len(s) == 20 and s[0] == np.float32(1.01) and s[10] == np.float32(0.99)
    b = datagen.batch_sizes(0)
    assert len(b) == 64 and b.min() >= 10000 and b.max() <= 5_000_000
    qs = datagen.draw_queries(1, 200)
    arr = np.array([q.arrival for q in qs])
    assert np.all(np.diff(arr) > 0) and abs(200 / arr[-1] - 50) < 10
    assert all(15 <= q.mu_pt <= 40 and 25 <= q.jet_pt <= 60 and 2 <= q.min_jet <= 6 for q in qs)
    assert all(50 <= len(q.edges_ht) - 1 <= 200 for q in qs)
