// Host-side state of a fused-pass plan, shared by the translation units
// that build and launch plans (library internal, not part of the ABI).
#pragma once

#include <vector>

#include "pipeline_kernel.hpp"

struct hepk_plan_s {
    int device = 0;
    int32_t n_ds = 0, n_q = 0;
    int dtype = HEPK_F32;
    bool ext = false;
    bool shared = false;
    bool ms = false;  // some query slot holds several jet-energy scales
    bool lk = false;  // lookup-correction kernels (queries with lookups, or sums of squared weights)
    hepk_tune tune{};
    int grid = 0;
    hepk::KernelFn fn_lds = nullptr, fn_glob = nullptr;
    hepk::KernelFn fn_lds_dbg = nullptr, fn_glob_dbg = nullptr;  // with per-event records
    bool dbg_ok = false;               // record kernels have the product kernels' LDS
    std::vector<int64_t> ev_pre;       // n_ds + 1: events of the datasets before each
    size_t lds_static_lds = 0, lds_static_glob = 0;  // static LDS of the two kernels
    size_t lds_max = 0;                              // the device's LDS per workgroup
    hepk::PipeArgs args{};             // table pointers; chunk range and histograms set per launch
    std::vector<int64_t> tile_pre;     // n_ds + 1: tiles of the datasets before each (chunk d = dataset d)
    int64_t ds_block = 0;              // histogram slots per dataset block
    int64_t n_slots = 0;
    std::vector<hepk::QDev> qd;        // host copy of the query table
    std::vector<int32_t> cap_bins;     // (slot, h): reserved bins
    std::vector<int32_t> cap_scales;   // slot: reserved scales
    int32_t lds_slots = 0;             // LDS histogram slots of the active queries
    int32_t n_edges = 0, n_scales = 0;
    bool edges_lds = false, scales_lds = false;
    void *dev_mem = nullptr;
    hepk::QDev *d_q = nullptr;
    float *d_scales = nullptr, *d_edges = nullptr;
    // pinned staging ring for hepk_plan_set_query
    char *pinned = nullptr;
    size_t stage_bytes = 0;
    int ring_pos = 0;
    std::vector<hipEvent_t> ring_ev;
    std::vector<bool> ring_used;
    // graph launch
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipGraphNode_t gnode = nullptr;
    hepk::KernelFn gfn = nullptr;
    hepk::PipeArgs gargs{};
    size_t glds = 0;
    int ggrid = 0;
};

namespace hepk {

// Offsets of the tables in the one block of device memory the kernels read.
struct TableLayout {
    size_t o_ds, o_ch, o_q, o_sc, o_e, total;
    int32_t max_cap, max_sc;  // largest reserved bins and scales of a slot
};

// One launch of the fused kernel.
struct Launch {
    KernelFn fn;
    int grid, block;
    size_t lds;         // dynamic LDS
    size_t lds_static;  // the kernel's static LDS
    size_t lds_max;
    PipeArgs a;
};

// Validates the datasets and queries and builds a plan's host state and the
// image of its device tables (img, laid out as lay), without touching device
// memory.  On success *out owns the new plan (release with free_plan).
int plan_build(const hepk_dataset *ds, int32_t n_ds, const hepk_query *q, int32_t n_query,
               const hepk_plan_opts *opts, hepk_plan *out, std::vector<char> &img, TableLayout &lay);

// Points the plan's launch arguments at its tables, copied to device memory
// at base (laid out as lay).
void plan_bind(hepk_plan p, char *base, const TableLayout &lay);

// The launch over chunks [c0, c1) (per-event records into rec when not NULL,
// squared weights into sumw2 when not NULL: lookup plans only).
Launch make_launch(hepk_plan p, int32_t c0, int32_t c1, double *sumw, uint64_t *counts,
                   hepk_event_record *rec = nullptr, double *sumw2 = nullptr);

// Checks the launch's LDS against the device's and enqueues it.
int run_launch(const Launch &L, hipStream_t stream);

// Datasets [c0, c1) have work and some query slot is active.
bool has_work(hepk_plan p, int32_t c0, int32_t c1);

// Releases everything the plan holds.
void free_plan(hepk_plan p);

}  // namespace hepk
