// hepk_reduce: per-event segmented reductions over jagged content
// (Sec. III: the H_T kernel of Listing 1 and the count/sum/max/min-within-
// offsets kernels).
//
// A workgroup takes a tile of RB consecutive events.  Their objects form one
// contiguous content range, which is staged through LDS in chunks of RCH with
// coalesced loads; then one lane per event walks its own objects in order.
// Walking in order keeps the float32 sum identical to the left-to-right sum
// of Listing 1's inner loop (a tree would round differently), and gives the
// lowest index on max/min ties.  Counts feed an optional exclusive scan that
// yields the offsets of the selected sub-collection.
#include "common.hpp"

namespace hepk {

constexpr int RB = 256;    // events per tile == threads per workgroup
constexpr int RCH = 4096;  // objects staged per chunk

enum { R_COUNT = 0, R_SUM = 1, R_MAX = 2, R_MIN = 3 };

// Inclusive scan of one int64 per thread over a workgroup of RB threads.
__device__ int64_t block_inclusive_scan(int64_t v, int64_t *buf) {
    const int tid = threadIdx.x;
    buf[tid] = v;
    __syncthreads();
    for (int d = 1; d < RB; d <<= 1) {
        int64_t add = (tid >= d) ? buf[tid - d] : 0;
        __syncthreads();
        v += add;
        buf[tid] = v;
        __syncthreads();
    }
    return v;
}

template <typename T, int OP>
__global__ __launch_bounds__(RB) void reduce_kernel(const int64_t *__restrict__ off, int64_t n_events,
                                                    const T *__restrict__ content,
                                                    const uint8_t *__restrict__ obj_mask,
                                                    const uint8_t *__restrict__ evt_mask, void *out,
                                                    int32_t *out_arg, int index_only, int64_t *tile_tot) {
    __shared__ int64_t off_s[RB + 1];
    __shared__ float val_s[(OP == R_COUNT) ? 1 : RCH];
    __shared__ uint8_t msk_s[RCH];
    __shared__ int64_t scan_s[RB];
    const int tid = threadIdx.x;
    const int64_t n_tiles = ceil_div(n_events, RB);
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t e0 = tile * RB;
        const int ne = static_cast<int>(n_events - e0 < RB ? n_events - e0 : RB);
        const int64_t A = off[e0];
        const int64_t B = off[e0 + ne];
        if (tid < ne) off_s[tid] = off[e0 + tid] - A;
        if (tid == 0) off_s[ne] = B - A;
        __syncthreads();
        const bool act = tid < ne;
        const int64_t e = e0 + tid;
        const bool take = act && (!evt_mask || evt_mask[e] != 0);
        const int64_t a0 = act ? off_s[tid] : 0;
        const int64_t a1 = act ? off_s[tid + 1] : 0;
        int32_t cnt = 0;
        float acc = 0.0f;
        float best = (OP == R_MAX) ? -INFINITY : INFINITY;
        int32_t bi = -1;
        if (OP == R_COUNT && !obj_mask) {
            cnt = take ? static_cast<int32_t>(a1 - a0) : 0;
        } else {
            const int64_t tot = B - A;
            for (int64_t c0 = 0; c0 < tot; c0 += RCH) {
                const int clen = static_cast<int>(tot - c0 < RCH ? tot - c0 : RCH);
                for (int i = tid; i < clen; i += RB) {
                    if (OP != R_COUNT) val_s[i] = ldf(content, A + c0 + i);
                    msk_s[i] = obj_mask ? obj_mask[A + c0 + i] : 1;
                }
                __syncthreads();
                if (take) {
                    const int64_t k0 = a0 > c0 ? a0 : c0;
                    const int64_t k1 = a1 < c0 + clen ? a1 : c0 + clen;
                    for (int64_t k = k0; k < k1; ++k) {
                        const int kk = static_cast<int>(k - c0);
                        if (!msk_s[kk]) continue;
                        if (OP == R_COUNT) {
                            ++cnt;
                        } else if (OP == R_SUM) {
                            acc = acc + val_s[kk];
                        } else {
                            const float v = val_s[kk];
                            const bool better = (OP == R_MAX) ? (v > best) : (v < best);
                            if (bi < 0 || better) {
                                best = v;
                                bi = static_cast<int32_t>(k - a0);
                            }
                        }
                    }
                }
                __syncthreads();
            }
        }
        if (act) {
            if (OP == R_COUNT) {
                static_cast<int32_t *>(out)[e] = cnt;
            } else if (OP == R_SUM) {
                static_cast<float *>(out)[e] = acc;
            } else if (index_only) {
                static_cast<int32_t *>(out)[e] = bi;
            } else {
                static_cast<float *>(out)[e] = best;
                if (out_arg) out_arg[e] = bi;
            }
        }
        if (OP == R_COUNT && tile_tot) {
            int64_t incl = block_inclusive_scan(act ? cnt : 0, scan_s);
            if (tid == RB - 1) tile_tot[tile] = incl;
        }
        __syncthreads();
    }
}

// Exclusive scan, in place, of n int64 values by one workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void scan_tiles_kernel(int64_t *v, int64_t n) {
    __shared__ int64_t buf[1024];
    const int tid = threadIdx.x;
    const int64_t per = ceil_div(n, 1024);
    const int64_t b = tid * per;
    const int64_t e = (b + per < n) ? b + per : n;
    int64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += v[i];
    buf[tid] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        int64_t add = (tid >= d) ? buf[tid - d] : 0;
        __syncthreads();
        buf[tid] += add;
        __syncthreads();
    }
    int64_t run = buf[tid] - s;  // exclusive prefix of this thread's chunk
    for (int64_t i = b; i < e; ++i) {
        int64_t x = v[i];
        v[i] = run;
        run += x;
    }
}

// offsets_out[0] = 0, offsets_out[e+1] = sum of counts[0..e].
__global__ __launch_bounds__(RB) void offsets_from_counts_kernel(const int32_t *counts, int64_t n_events,
                                                                 const int64_t *tile_pre, int64_t *offsets_out) {
    __shared__ int64_t scan_s[RB];
    const int tid = threadIdx.x;
    const int64_t n_tiles = ceil_div(n_events, RB);
    if (blockIdx.x == 0 && tid == 0) offsets_out[0] = 0;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t e = tile * RB + tid;
        const int64_t c = (e < n_events) ? counts[e] : 0;
        const int64_t incl = block_inclusive_scan(c, scan_s);
        if (e < n_events) offsets_out[e + 1] = tile_pre[tile] + incl;
        __syncthreads();
    }
}

template <typename T, int OP>
static int launch_reduce(const int64_t *off, int64_t n, const void *content, const uint8_t *om,
                         const uint8_t *em, void *out, int32_t *out_arg, int index_only, int64_t *tile_tot,
                         hipStream_t stream) {
    const int64_t n_tiles = ceil_div(n, RB);
    const int grid = static_cast<int>(std::min<int64_t>(n_tiles, 8 * device_cus()));
    reduce_kernel<T, OP><<<grid, RB, 0, stream>>>(off, n, static_cast<const T *>(content), om, em, out,
                                                  out_arg, index_only, tile_tot);
    return check_launch("hepk_reduce");
}

}  // namespace hepk

extern "C" int hepk_reduce(int32_t op, const int64_t *offsets, int64_t n_events, const void *content,
                           int32_t dtype, const uint8_t *obj_mask, const uint8_t *evt_mask, void *out,
                           int32_t *out_arg, int64_t *offsets_out, hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(op >= HEPK_COUNT && op <= HEPK_ARGMIN, "hepk_reduce: bad op %d", op);
    HEPK_REQUIRE(n_events >= 0, "hepk_reduce: n_events < 0");
    HEPK_REQUIRE(offsets, "hepk_reduce: offsets is NULL");
    HEPK_REQUIRE(n_events == 0 || out, "hepk_reduce: out is NULL");
    HEPK_REQUIRE(!offsets_out || op == HEPK_COUNT, "hepk_reduce: offsets_out is for COUNT only");
    HEPK_REQUIRE(!out_arg || op == HEPK_MAX || op == HEPK_MIN, "hepk_reduce: out_arg is for MAX/MIN only");
    if (op != HEPK_COUNT) {
        if (dtype != HEPK_F32 && dtype != HEPK_F16) {
            set_error("hepk_reduce: content dtype %d unsupported for this op", dtype);
            return HEPK_EUNSUPPORTED;
        }
        HEPK_REQUIRE(content || n_events == 0, "hepk_reduce: content is NULL");
    }
    if (n_events == 0) {
        if (offsets_out) {  // writes offsets_out[0] = 0 only
            offsets_from_counts_kernel<<<1, RB, 0, stream>>>(nullptr, 0, nullptr, offsets_out);
            return check_launch("hepk_reduce offsets");
        }
        return HEPK_OK;
    }
    int64_t *tile_tot = nullptr;
    const int64_t n_tiles = ceil_div(n_events, RB);
    if (offsets_out) {
        hipError_t e = hipMallocAsync(reinterpret_cast<void **>(&tile_tot), n_tiles * sizeof(int64_t), stream);
        if (e != hipSuccess) {
            set_error("hepk_reduce: temporary of %lld bytes: %s", (long long)(n_tiles * 8), hipGetErrorString(e));
            return HEPK_ENOMEM;
        }
    }
    int rc;
    const bool h = dtype == HEPK_F16;
    switch (op) {
    case HEPK_COUNT:
        rc = launch_reduce<float, R_COUNT>(offsets, n_events, nullptr, obj_mask, evt_mask, out, nullptr, 0,
                                           tile_tot, stream);
        break;
    case HEPK_SUM:
        rc = h ? launch_reduce<_Float16, R_SUM>(offsets, n_events, content, obj_mask, evt_mask, out, nullptr, 0,
                                                nullptr, stream)
               : launch_reduce<float, R_SUM>(offsets, n_events, content, obj_mask, evt_mask, out, nullptr, 0,
                                             nullptr, stream);
        break;
    case HEPK_MAX:
    case HEPK_ARGMAX:
        rc = h ? launch_reduce<_Float16, R_MAX>(offsets, n_events, content, obj_mask, evt_mask, out, out_arg,
                                                op == HEPK_ARGMAX, nullptr, stream)
               : launch_reduce<float, R_MAX>(offsets, n_events, content, obj_mask, evt_mask, out, out_arg,
                                             op == HEPK_ARGMAX, nullptr, stream);
        break;
    default:
        rc = h ? launch_reduce<_Float16, R_MIN>(offsets, n_events, content, obj_mask, evt_mask, out, out_arg,
                                                op == HEPK_ARGMIN, nullptr, stream)
               : launch_reduce<float, R_MIN>(offsets, n_events, content, obj_mask, evt_mask, out, out_arg,
                                             op == HEPK_ARGMIN, nullptr, stream);
        break;
    }
    if (rc == HEPK_OK && offsets_out) {
        scan_tiles_kernel<<<1, 1024, 0, stream>>>(tile_tot, n_tiles);
        rc = check_launch("hepk_reduce scan");
        if (rc == HEPK_OK) {
            const int grid = static_cast<int>(std::min<int64_t>(n_tiles, 8 * device_cus()));
            offsets_from_counts_kernel<<<grid, RB, 0, stream>>>(static_cast<const int32_t *>(out), n_events,
                                                                tile_tot, offsets_out);
            rc = check_launch("hepk_reduce offsets");
        }
    }
    if (tile_tot) {
        hipError_t e = hipFreeAsync(tile_tot, stream);
        if (rc == HEPK_OK && e != hipSuccess) {
            set_error("hepk_reduce: hipFreeAsync: %s", hipGetErrorString(e));
            rc = HEPK_EHIP;
        }
    }
    return rc;
}
