// libhepk runtime pieces: per-thread error text, device properties, the
// ABI version and the offsets validator.
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace hepk {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

int check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_error("%s launch failed: %s", what, hipGetErrorString(e));
        return HEPK_EHIP;
    }
    return HEPK_OK;
}

int device_cus() {
    static std::mutex mu;
    static std::vector<int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> lk(mu);
    if (dev >= static_cast<int>(cache.size())) cache.resize(dev + 1, 0);
    if (cache[dev] == 0) {
        int n = 0;
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        cache[dev] = n;
    }
    return cache[dev];
}

// Counts offsets[0] != 0, offsets[i+1] < offsets[i] and offsets[N] != M.
__global__ void validate_offsets_kernel(const int64_t *off, int64_t n, int64_t m,
                                        unsigned long long *bad) {
    unsigned long long local = 0;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        local += (off[i + 1] < off[i]) ? 1ull : 0ull;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        local += (off[0] != 0) ? 1ull : 0ull;
        local += (off[n] != m) ? 1ull : 0ull;
    }
    if (local) atomicAdd(bad, local);
}

__global__ void zero_i64_kernel(int64_t *p) { *p = 0; }

// Grid-stride read of n16 16-byte words: eight nontemporal loads in flight
// per thread (the data is read once, so the loads ask the caches not to keep
// it), one 256-thread workgroup per compute unit -- the fastest of the block
// sizes (256-1024), loads in flight (4-16), grids (1-32 workgroups per
// compute unit) and cache hints measured on MI355X.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kStreamUnroll = 8;

__global__ __launch_bounds__(256) void stream_read_kernel(const u32x4 *__restrict__ p, int64_t n16, uint32_t key,
                                                          uint32_t *sink) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
    int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    uint32_t acc = 0;
    for (; i + (kStreamUnroll - 1) * stride < n16; i += kStreamUnroll * stride) {
        u32x4 v[kStreamUnroll];
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) v[u] = __builtin_nontemporal_load(p + i + u * stride);
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; i < n16; i += stride) {
        const u32x4 v = __builtin_nontemporal_load(p + i);
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    // data-dependent (the compiler cannot drop the loads); a match, should the
    // data ever give one, only writes the caller's sink
    if (acc == key) *sink = acc;
}

}  // namespace hepk

extern "C" const char *hepk_last_error(void) { return hepk::g_err; }

extern "C" int hepk_abi_version(void) { return HEPK_ABI_VERSION; }

extern "C" int hepk_validate_offsets(const int64_t *offsets, int64_t n_events, int64_t n_objects,
                                     int64_t *bad, hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(offsets && bad, "hepk_validate_offsets: null pointer");
    HEPK_REQUIRE(n_events >= 0 && n_objects >= 0, "hepk_validate_offsets: negative size");
    zero_i64_kernel<<<1, 1, 0, stream>>>(bad);
    int grid = static_cast<int>(std::min<int64_t>(std::max<int64_t>(1, ceil_div(n_events, 256)), 4 * device_cus()));
    validate_offsets_kernel<<<grid, 256, 0, stream>>>(offsets, n_events, n_objects,
                                                      reinterpret_cast<unsigned long long *>(bad));
    return check_launch("hepk_validate_offsets");
}

extern "C" int hepk_stream_read(const void *p, int64_t nbytes, uint32_t *sink, hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(p && sink, "hepk_stream_read: null pointer");
    HEPK_REQUIRE(nbytes >= 0 && nbytes % 16 == 0, "hepk_stream_read: nbytes %lld not a multiple of 16",
                 (long long)nbytes);
    HEPK_REQUIRE(reinterpret_cast<uintptr_t>(p) % 16 == 0, "hepk_stream_read: p not 16-byte aligned");
    if (nbytes == 0) return HEPK_OK;
    const int64_t n16 = nbytes / 16;
    const int grid = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(ceil_div(n16, 256 * kStreamUnroll),
                                                                            device_cus())));
    stream_read_kernel<<<grid, 256, 0, stream>>>(static_cast<const u32x4 *>(p), n16, 0x9e3779b9u, sink);
    return check_launch("hepk_stream_read");
}
