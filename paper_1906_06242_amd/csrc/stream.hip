// Out-of-core analysis passes (Sec. II: a cache of uncompressed columns in
// host memory or memory-mapped files; Fig. 1: the cache is loaded in batches
// of a few GB of contiguous arrays with the kernels dispatched on device
// memory).
//
// A streamer holds n_buffers device staging slots (and, for sources in
// pageable memory such as memory-mapped files, as many pinned host slots).
// A pass cuts the host dataset into batches of consecutive events and, for
// batch k in slot k % n_buffers:
//   host   waits until the slot's previous copy has left its pinned slot,
//          gathers the batch's columns into it with several threads (sources
//          already pinned are copied from directly), builds the batch's plan
//          tables;
//   copy   (the streamer's own stream) waits until the slot's previous pass
//          has finished reading it, then moves the columns and tables to the
//          device slot;
//   compute (the caller's stream) waits for that copy and runs the fused
//          pass on the batch, accumulating into the caller's histograms.
// So the copy of batch k+1 (DMA engine) and the host gathering of batch k+2
// overlap the pass over batch k.  Offsets stay absolute: a batch's offsets
// are the slice [e0, e1] of the host offsets, and its content pointers are
// placed so that content index off[e] lands on the slot's copy.
#include <algorithm>
#include <cstring>
#include <thread>
#include <vector>

#include "plan.hpp"

namespace hepk {

// One column of the host dataset: source pointer, element size, and whether
// it is indexed by objects of a collection (0 jets, 1 muons, 2 electrons) or
// by events (-1) or is an offsets array (3 + collection).
struct HostCol {
    const char *src;
    int es;
    int kind;
    const void **dev_field;  // where the batch dataset's device pointer goes
};

struct Batch {
    int64_t e0, e1;
    int64_t o0[3], o1[3];  // object ranges of jets, muons, electrons
};

}  // namespace hepk

struct hepk_streamer_s {
    int device = 0;
    hepk_dataset host{};  // host pointers
    std::vector<hepk_query> q;  // copies of the structs (their host arrays stay the caller's)
    hepk_plan_opts opts{};
    int n_buf = 2;
    size_t slot_bytes = 0;   // device (and pinned) bytes of one slot's columns
    size_t table_bytes = 0;  // bytes reserved for one batch's plan tables
    std::vector<hepk::Batch> batches;
    std::vector<char *> dev, pin;  // per slot
    bool src_pinned = false;
    hipStream_t copy = nullptr;
    std::vector<hipEvent_t> copied, done;
    std::vector<bool> used;
    int threads = 1;
    int64_t n_slots = 0;  // histogram slots
};

namespace hepk {

static size_t al256(size_t x) { return (x + 255) & ~size_t(255); }

static bool host_pinned(const void *p) {
    if (!p) return true;
    hipPointerAttribute_t a{};
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();  // pageable memory is not known to HIP
        return false;
    }
    return a.type == hipMemoryTypeHost;
}

// The columns of a dataset, with the device-pointer fields of `dst` they fill.
static std::vector<HostCol> columns(const hepk_dataset &h, hepk_dataset &dst) {
    const int es = h.dtype == HEPK_F16 ? 2 : 4;
    std::vector<HostCol> c;
    auto coll = [&](const hepk_collection &src, hepk_collection &d, int k) {
        if (!src.offsets) return;
        c.push_back({reinterpret_cast<const char *>(src.offsets), 8, 3 + k,
                     reinterpret_cast<const void **>(&d.offsets)});
        c.push_back({static_cast<const char *>(src.pt), es, k, &d.pt});
        c.push_back({static_cast<const char *>(src.eta), es, k, &d.eta});
        c.push_back({static_cast<const char *>(src.phi), es, k, &d.phi});
        if (src.extra) c.push_back({static_cast<const char *>(src.extra), es, k, &d.extra});
    };
    coll(h.jets, dst.jets, 0);
    coll(h.muons, dst.muons, 1);
    coll(h.electrons, dst.electrons, 2);
    if (h.weights)
        c.push_back({reinterpret_cast<const char *>(h.weights), 4, -1, reinterpret_cast<const void **>(&dst.weights)});
    if (h.npu) c.push_back({reinterpret_cast<const char *>(h.npu), 4, -1, reinterpret_cast<const void **>(&dst.npu)});
    return c;
}

// Bytes of one column's slice for a batch (256-byte aligned).
static size_t slice_bytes(const HostCol &c, const Batch &b) {
    if (c.kind == -1) return al256(static_cast<size_t>(b.e1 - b.e0) * c.es);
    if (c.kind >= 3) return al256(static_cast<size_t>(b.e1 - b.e0 + 1) * c.es);
    return al256(static_cast<size_t>(std::max<int64_t>(1, b.o1[c.kind] - b.o0[c.kind])) * c.es);
}

static int64_t first_index(const HostCol &c, const Batch &b) {
    return c.kind >= 0 && c.kind < 3 ? b.o0[c.kind] : b.e0;
}

static int64_t count(const HostCol &c, const Batch &b) {
    if (c.kind == -1) return b.e1 - b.e0;
    if (c.kind >= 3) return b.e1 - b.e0 + 1;
    return b.o1[c.kind] - b.o0[c.kind];
}

// Copies n bytes with up to `threads` threads.
static void par_copy(char *dst, const char *src, size_t n, int threads) {
    constexpr size_t kMinPerThread = size_t(8) << 20;
    const int t = static_cast<int>(std::min<size_t>(threads, std::max<size_t>(1, n / kMinPerThread)));
    if (t <= 1) {
        std::memcpy(dst, src, n);
        return;
    }
    std::vector<std::thread> ws;
    const size_t per = (n + t - 1) / t;
    for (int i = 0; i < t; ++i) {
        const size_t a = i * per, z = std::min(n, a + per);
        if (a < z) ws.emplace_back([=] { std::memcpy(dst + a, src + a, z - a); });
    }
    for (auto &w : ws) w.join();
}

static void free_streamer(hepk_streamer s) {
    if (!s) return;
    for (size_t i = 0; i < s->copied.size(); ++i)
        if (s->used[i]) {
            (void)hipEventSynchronize(s->copied[i]);
            (void)hipEventSynchronize(s->done[i]);
        }
    for (auto e : s->copied) (void)hipEventDestroy(e);
    for (auto e : s->done) (void)hipEventDestroy(e);
    if (s->copy) (void)hipStreamDestroy(s->copy);
    for (auto p : s->dev) (void)hipFree(p);
    for (auto p : s->pin) (void)hipHostFree(p);
    delete s;
}

}  // namespace hepk

extern "C" int hepk_streamer_create(const hepk_dataset *host_ds, const hepk_query *q, int32_t n_query,
                                    const hepk_stream_opts *opts, hepk_streamer *out) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(out && host_ds && q && n_query >= 1, "hepk_streamer_create: NULL argument");
    *out = nullptr;
    hepk_stream_opts so{};
    if (opts) so = *opts;
    HEPK_REQUIRE(so.batch_events >= 0, "hepk_streamer_create: batch_events < 0");
    HEPK_REQUIRE(so.n_buffers == 0 || (so.n_buffers >= 1 && so.n_buffers <= 8),
                 "hepk_streamer_create: n_buffers %d not in [1, 8]", so.n_buffers);
    HEPK_REQUIRE(so.host_threads >= 0 && so.host_threads <= 64, "hepk_streamer_create: host_threads out of range");
    const hepk_dataset &H = *host_ds;
    HEPK_REQUIRE(H.n_events >= 0 && H.jets.offsets && H.muons.offsets, "hepk_streamer_create: bad dataset");
    hepk_streamer s = new hepk_streamer_s();
    s->host = H;
    s->n_buf = so.n_buffers ? so.n_buffers : 2;
    s->threads = so.host_threads ? so.host_threads : 8;
    s->opts.tune = so.tune;
    // copies of the queries (their host tables are read again for every batch)
    s->q.assign(q, q + n_query);
    if (hipGetDevice(&s->device) != hipSuccess) {
        set_error("hepk_streamer_create: no current HIP device");
        free_streamer(s);
        return HEPK_EHIP;
    }
    // batches of batch_events events (default 2^22)
    const int64_t be = so.batch_events ? so.batch_events : (int64_t(1) << 22);
    const hepk_collection *cs[3] = {&H.jets, &H.muons, &H.electrons};
    for (int64_t e0 = 0; e0 < H.n_events; e0 += be) {
        Batch b{};
        b.e0 = e0;
        b.e1 = std::min(H.n_events, e0 + be);
        for (int k = 0; k < 3; ++k) {
            b.o0[k] = cs[k]->offsets ? cs[k]->offsets[b.e0] : 0;
            b.o1[k] = cs[k]->offsets ? cs[k]->offsets[b.e1] : 0;
        }
        s->batches.push_back(b);
    }
    // slot size: the largest batch's columns, plus its plan tables
    hepk_dataset scratch{};
    const std::vector<HostCol> cols = columns(H, scratch);
    for (const Batch &b : s->batches) {
        size_t t = 0;
        for (const HostCol &c : cols) t += slice_bytes(c, b);
        s->slot_bytes = std::max(s->slot_bytes, t);
    }
    s->table_bytes = size_t(1) << 20;
    s->src_pinned = true;
    for (const HostCol &c : cols) s->src_pinned = s->src_pinned && host_pinned(c.src);
    const size_t total = s->slot_bytes + s->table_bytes;
    s->dev.assign(s->n_buf, nullptr);
    s->pin.assign(s->n_buf, nullptr);
    s->copied.assign(s->n_buf, nullptr);
    s->done.assign(s->n_buf, nullptr);
    s->used.assign(s->n_buf, false);
    int rc = HEPK_OK;
    for (int i = 0; i < s->n_buf && rc == HEPK_OK; ++i) {
        if (hipMalloc(&s->dev[i], total) != hipSuccess) {
            set_error("hepk_streamer_create: hipMalloc of %zu bytes failed", total);
            rc = HEPK_ENOMEM;
        } else if (hipHostMalloc(reinterpret_cast<void **>(&s->pin[i]), s->src_pinned ? s->table_bytes : total,
                                 hipHostMallocDefault) != hipSuccess) {
            set_error("hepk_streamer_create: pinned allocation failed");
            rc = HEPK_ENOMEM;
        } else if (hipEventCreateWithFlags(&s->copied[i], hipEventDisableTiming) != hipSuccess ||
                   hipEventCreateWithFlags(&s->done[i], hipEventDisableTiming) != hipSuccess) {
            set_error("hepk_streamer_create: event creation failed");
            rc = HEPK_EHIP;
        }
    }
    if (rc == HEPK_OK && hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) != hipSuccess) {
        set_error("hepk_streamer_create: copy stream creation failed");
        rc = HEPK_EHIP;
    }
    // the histogram layout (that of a plan over one batch), and a check that
    // the queries and launch configuration are valid
    if (rc == HEPK_OK) {
        std::vector<char> img;
        TableLayout lay{};
        hepk_plan p = nullptr;
        hepk_dataset d0 = H;
        d0.n_events = 0;
        rc = plan_build(&d0, 1, s->q.data(), n_query, &s->opts, &p, img, lay);
        if (rc == HEPK_OK) {
            s->n_slots = p->n_slots;
            free_plan(p);
        }
    }
    if (rc != HEPK_OK) {
        free_streamer(s);
        return rc;
    }
    *out = s;
    return HEPK_OK;
}

extern "C" int hepk_streamer_hist_slots(hepk_streamer s, int64_t *n_slots) {
    hepk::clear_error();
    HEPK_REQUIRE(s && n_slots, "hepk_streamer_hist_slots: NULL argument");
    *n_slots = s->n_slots;
    return HEPK_OK;
}

extern "C" int hepk_stream_pass(hepk_streamer s, double *sumw, uint64_t *counts, hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(s && sumw && counts, "hepk_stream_pass: NULL argument");
    int dev = 0;
    HEPK_HIP(hipGetDevice(&dev));
    HEPK_REQUIRE(dev == s->device, "hepk_stream_pass: streamer made on device %d, current device %d", s->device,
                 dev);
    for (size_t k = 0; k < s->batches.size(); ++k) {
        const Batch &b = s->batches[k];
        const int slot = static_cast<int>(k % s->n_buf);
        char *dbase = s->dev[slot];
        char *pbase = s->pin[slot];
        // the slot's pinned memory is free once its previous copy has run
        if (s->used[slot]) HEPK_HIP(hipEventSynchronize(s->copied[slot]));
        // the batch's dataset: device pointers into the slot, content placed
        // so that absolute object indices land on the slice
        hepk_dataset d = s->host;
        d.n_events = b.e1 - b.e0;
        const std::vector<HostCol> cols = columns(s->host, d);
        size_t at = 0;
        struct Piece {
            size_t at, bytes;
            const char *src;
        };
        std::vector<Piece> pieces;
        for (const HostCol &c : cols) {
            const int64_t first = first_index(c, b);
            const size_t nb = static_cast<size_t>(count(c, b)) * c.es;
            pieces.push_back({at, nb, c.src + static_cast<size_t>(first) * c.es});
            char *p = dbase + at;
            // offsets arrays and per-event columns start at the batch's
            // first event; content columns are indexed by absolute object
            if (c.kind >= 3 || c.kind == -1)
                *c.dev_field = p;
            else
                *c.dev_field = p - static_cast<size_t>(first) * c.es;
            at += slice_bytes(c, b);
        }
        std::vector<char> img;
        TableLayout lay{};
        hepk_plan p = nullptr;
        if (int rc = plan_build(&d, 1, s->q.data(), static_cast<int32_t>(s->q.size()), &s->opts, &p, img, lay))
            return rc;
        if (lay.total > s->table_bytes) {
            free_plan(p);
            set_error("hepk_stream_pass: plan tables of %zu bytes exceed the slot's %zu", lay.total, s->table_bytes);
            return HEPK_EINVAL;
        }
        // gather into pinned memory (pageable sources) and copy on the copy
        // stream once the slot's previous pass is done with it
        char *tpin = s->src_pinned ? pbase : pbase + s->slot_bytes;
        std::memcpy(tpin, img.data(), lay.total);
        int rc = HEPK_OK;
        if (s->used[slot] && hipStreamWaitEvent(s->copy, s->done[slot], 0) != hipSuccess) rc = HEPK_EHIP;
        for (const Piece &pc : pieces) {
            if (rc) break;
            const char *src = pc.src;
            if (!s->src_pinned) {
                par_copy(pbase + pc.at, pc.src, pc.bytes, s->threads);
                src = pbase + pc.at;
            }
            if (pc.bytes && hipMemcpyAsync(dbase + pc.at, src, pc.bytes, hipMemcpyHostToDevice, s->copy) != hipSuccess)
                rc = HEPK_EHIP;
        }
        char *dtab = dbase + s->slot_bytes;
        if (rc == HEPK_OK &&
            hipMemcpyAsync(dtab, tpin, lay.total, hipMemcpyHostToDevice, s->copy) != hipSuccess)
            rc = HEPK_EHIP;
        if (rc == HEPK_OK && hipEventRecord(s->copied[slot], s->copy) != hipSuccess) rc = HEPK_EHIP;
        if (rc == HEPK_OK && hipStreamWaitEvent(stream, s->copied[slot], 0) != hipSuccess) rc = HEPK_EHIP;
        if (rc == HEPK_OK) {
            plan_bind(p, dtab, lay);
            if (has_work(p, 0, 1)) rc = run_launch(make_launch(p, 0, 1, sumw, counts), stream);
        }
        if (rc == HEPK_OK && hipEventRecord(s->done[slot], stream) != hipSuccess) rc = HEPK_EHIP;
        free_plan(p);
        if (rc == HEPK_EHIP) set_error("hepk_stream_pass: a copy, event or launch call failed on batch %zu", k);
        if (rc) return rc;
        s->used[slot] = true;
    }
    return HEPK_OK;
}

extern "C" int hepk_streamer_destroy(hepk_streamer s) {
    hepk::clear_error();
    hepk::free_streamer(s);
    return HEPK_OK;
}
