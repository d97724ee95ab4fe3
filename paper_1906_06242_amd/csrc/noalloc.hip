// hepk_pipeline_noalloc: the fused pass for callers that cannot allocate
// device memory.  The plan's device tables (datasets, work chunks, queries,
// scales, bin edges) go into a fixed file-scope device array instead of a
// hipMalloc'd block; everything else is the path of hepk_plan_create +
// hepk_pipeline (same kernels, same launch configuration).
#include <mutex>
#include <vector>

#include "plan.hpp"

namespace hepk {

constexpr size_t kNoAllocScratchBytes = size_t(1) << 20;

// One copy per device, held until the process ends.  Host code never uses
// this name as an address: it holds a host-side stand-in, so only the device
// address from hipGetSymbolAddress is passed to copies and kernels.
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

// The device address of `scratch` on the current device (looked up once per
// device, with that device current).
static int scratch_address(int dev, char **out) {
    static std::mutex mu;
    static std::vector<char *> addr;
    std::lock_guard<std::mutex> lk(mu);
    if (dev >= static_cast<int>(addr.size())) addr.resize(dev + 1, nullptr);
    if (!addr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hepk_pipeline_noalloc: hipGetSymbolAddress failed: %s", hipGetErrorString(e));
            return HEPK_EHIP;
        }
        addr[dev] = static_cast<char *>(p);
    }
    *out = addr[dev];
    return HEPK_OK;
}

}  // namespace hepk

extern "C" int hepk_pipeline_noalloc(const hepk_dataset *ds, int32_t n_ds, const hepk_query *q, int32_t n_query,
                                     const hepk_tune *tune, double *sumw, uint64_t *counts, hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(sumw && counts, "hepk_pipeline_noalloc: histogram buffers are NULL");
    hepk_plan_opts o{};
    if (tune) {
        HEPK_REQUIRE(tune->block != 0, "hepk_pipeline_noalloc: tune.block 0 is not a launch shape");
        o.tune = *tune;
    }
    std::vector<char> img;
    TableLayout lay{};
    hepk_plan p = nullptr;
    if (int rc = plan_build(ds, n_ds, q, n_query, &o, &p, img, lay)) return rc;
    int rc = HEPK_OK;
    char *base = nullptr;
    if (lay.total > kNoAllocScratchBytes) {
        set_error("hepk_pipeline_noalloc: tables need %zu bytes, the fixed scratch holds %zu", lay.total,
                  kNoAllocScratchBytes);
        rc = HEPK_EINVAL;
    } else if ((rc = scratch_address(p->device, &base)) == HEPK_OK) {
        // stream-ordered: a launch enqueued earlier on this stream reads the
        // previous tables before they are overwritten
        const hipError_t e = hipMemcpyAsync(base, img.data(), lay.total, hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) {
            set_error("hepk_pipeline_noalloc: table upload failed: %s", hipGetErrorString(e));
            rc = HEPK_EHIP;
        } else {
            plan_bind(p, base, lay);
            if (has_work(p, 0, p->n_ds)) rc = run_launch(make_launch(p, 0, p->n_ds, sumw, counts), stream);
        }
    }
    free_plan(p);  // host state only: this plan holds no device memory
    return rc;
}
