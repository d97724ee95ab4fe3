// hepk_reduce: per-event segmented reductions over jagged content
// (Sec. III: the H_T kernel of Listing 1, the count/sum/max/min-within-
// offsets kernels, and the generic pairwise operator taken as the product).
//
// Each wavefront owns tiles of 64 consecutive events and works through them
// without waiting for the rest of its workgroup.  For one tile it reads the
// tile's object range with two scalar loads, then issues every load of the
// tile at once -- both offsets and the event mask of each event lane, and up
// to RK objects (content and object mask) per lane, consecutive lanes on
// consecutive objects -- stages the objects in its own LDS region, and lets
// one lane per event walk its objects in order.  Walking in order keeps the
// float32 sum identical to the left-to-right sum of Listing 1's inner loop (a
// tree would round differently), and gives the lowest index on max/min ties.
// A tile with more than 64 * RK objects is walked straight from HBM, one lane
// per event, with the same arithmetic.  Counts can feed an exclusive scan
// that yields the offsets of the selected sub-collection.
#include "common.hpp"

namespace hepk {

constexpr int RB = 256;  // threads per workgroup; events per tile of the offsets scan
constexpr int RW = RB / 64;
constexpr int RK = 8;    // objects per lane staged for one tile (512 per tile)

enum { R_COUNT = 0, R_SUM = 1, R_MAX = 2, R_MIN = 3, R_PROD = 4 };

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

__device__ __forceinline__ void wave_fence() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Running reduction of one event.
template <int OP>
struct Acc {
    int32_t cnt = 0;
    float sum = 0.0f;
    float prod = 1.0f;
    float best = (OP == R_MAX) ? -INFINITY : INFINITY;
    int32_t bi = -1;
    __device__ __forceinline__ void add(float v, bool keep, int32_t k) {
        if (!keep) return;
        if (OP == R_COUNT) {
            ++cnt;
        } else if (OP == R_SUM) {
            sum = sum + v;
        } else if (OP == R_PROD) {
            prod = prod * v;
        } else {
            const bool better = (OP == R_MAX) ? (v > best) : (v < best);
            if (bi < 0 || better) {
                best = v;
                bi = k;
            }
        }
    }
};

template <typename T, int OP>
__global__ __launch_bounds__(RB) void reduce_kernel(const int64_t *__restrict__ off, int64_t n_events,
                                                    const T *__restrict__ content,
                                                    const uint8_t *__restrict__ obj_mask,
                                                    const uint8_t *__restrict__ evt_mask, void *out,
                                                    int32_t *out_arg, int index_only) {
    static_assert(__is_same(T, float) || __is_same(T, _Float16), "content is float32 or float16 (raw_f)");
    __shared__ float val_s[RW][(OP == R_COUNT) ? 1 : 64 * RK];
    // the tile's mask bytes as the 4-byte words that hold them (the first
    // byte of the range at byte s of the first word)
    constexpr int RMW = (64 * RK + 3 + 255) / 256;  // words per lane
    __shared__ uint32_t msk_s[RW][64 * RMW];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float *vs = val_s[wave];
    uint32_t *msw = msk_s[wave];
    const int64_t n_tiles = ceil_div(n_events, 64);
    const bool walk_objects = !(OP == R_COUNT && !obj_mask);
    const int64_t step = static_cast<int64_t>(gridDim.x) * RW;
    // the object range of a tile is fetched one tile ahead (scalar loads that
    // overlap the current tile's work)
    auto bounds = [&](int64_t t, int64_t &lo, int64_t &hi) {
        const int64_t e0 = t * 64;
        lo = as_const(off)[e0];
        hi = as_const(off)[e0 + min<int64_t>(64, n_events - e0)];
    };
    int64_t t = static_cast<int64_t>(blockIdx.x) * RW + wave;
    int64_t nA = 0, nB = 0;
    if (t < n_tiles) bounds(t, nA, nB);
    for (; t < n_tiles; t += step) {
        const int64_t e0 = t * 64;
        const int ne = static_cast<int>(min<int64_t>(64, n_events - e0));
        const int64_t A = nA;
        const int64_t tot = nB - nA;
        if (t + step < n_tiles) bounds(t + step, nA, nB);
        const int64_t e = e0 + lane;
        const bool act = lane < ne;
        // the tile's loads are buffer loads over exactly its ranges (0 past
        // their ends: no per-lane or per-slot branch), waited for together:
        // both offsets of each event lane's event (their low 32-bit words:
        // tile-relative differences are exact modulo 2^32), its event mask
        // byte, and below the objects and their mask words
        const buf_t bo = buf_span(off + e0, static_cast<uint32_t>(ne + 1) * 8u);
        const uint32_t o0 = buf_u32(bo, lane * 8), o1 = buf_u32(bo, lane * 8 + 8);
        const buf_t bev = buf_span(evt_mask ? static_cast<const void *>(evt_mask + e0) : static_cast<const void *>(off),
                                   evt_mask ? static_cast<uint32_t>(ne) : 0u);
        const uint32_t evb = evt_mask ? __builtin_amdgcn_raw_buffer_load_b8(bev, lane, 0, 0) : 1u;
        int64_t a0 = 0, a1 = 0;  // the event's objects, relative to the tile's first
        bool take = false;
        auto event_range = [&]() {
            a0 = act ? static_cast<int32_t>(o0 - static_cast<uint32_t>(A)) : 0;
            a1 = act ? static_cast<int32_t>(o1 - static_cast<uint32_t>(A)) : 0;
            take = act && evb != 0u;
        };
        Acc<OP> r;
        if (!walk_objects) {
            event_range();
            r.cnt = take ? static_cast<int32_t>(a1 - a0) : 0;
        } else if (tot <= 64 * RK) {
            const int n = static_cast<int>(tot);
            const buf_t bc = buf_span(content + A, static_cast<uint32_t>(n) * sizeof(T));
            uint32_t rv[RK];
#pragma unroll
            for (int k = 0; k < RK; ++k) rv[k] = OP != R_COUNT ? buf_raw<T>(bc, lane + 64 * k) : 0u;
            // mask bytes in 4-byte loads: the aligned words that hold bytes
            // [A, A + n)
            int s = 0, nw = 0;
            uint32_t mw[RMW];
#pragma unroll
            for (int k = 0; k < RMW; ++k) mw[k] = 0u;
            if (obj_mask) {
                const uint8_t *p = obj_mask + A;
                s = static_cast<int>(reinterpret_cast<uintptr_t>(p) & 3u);
                nw = n > 0 ? (n + s + 3) >> 2 : 0;
                const buf_t bw = buf_span(p - s, static_cast<uint32_t>(nw) * 4u);
#pragma unroll
                for (int k = 0; k < RMW; ++k) mw[k] = buf_u32(bw, (lane + 64 * k) * 4);
            }
            asm volatile("" ::"v"(o0), "v"(o1), "v"(evb));
#pragma unroll
            for (int k = 0; k < RK; ++k) asm volatile("" ::"v"(rv[k]));
#pragma unroll
            for (int k = 0; k < RMW; ++k) asm volatile("" ::"v"(mw[k]));
            event_range();
            float v[RK];
#pragma unroll
            for (int k = 0; k < RK; ++k) v[k] = raw_f<T>(rv[k]);
#pragma unroll
            for (int k = 0; k < RK; ++k) {
                const int i = lane + 64 * k;
                if (OP != R_COUNT && i < n) vs[i] = v[k];
            }
            if (obj_mask) {
#pragma unroll
                for (int k = 0; k < RMW; ++k) {
                    const int w = lane + 64 * k;
                    if (w < nw) msw[w] = mw[k];
                }
            }
            const uint8_t *ms = reinterpret_cast<const uint8_t *>(msw) + s;
            const bool all = obj_mask == nullptr;
            wave_fence();
            const int b0 = static_cast<int>(a0), b1 = static_cast<int>(a1);  // within the tile's 512
            if (take) {
                // two objects per step (both LDS reads in flight), in order
                int k = b0;
                for (; k + 2 <= b1; k += 2) {
                    const float v0 = OP != R_COUNT ? vs[k] : 0.0f, v1 = OP != R_COUNT ? vs[k + 1] : 0.0f;
                    const bool m0 = all || ms[k] != 0, m1 = all || ms[k + 1] != 0;
                    r.add(v0, m0, k - b0);
                    r.add(v1, m1, k + 1 - b0);
                }
                if (k < b1) r.add(OP != R_COUNT ? vs[k] : 0.0f, all || ms[k] != 0, k - b0);
            }
            wave_fence();  // the next tile overwrites the staging
        } else if (event_range(), take) {
            for (int64_t k = a0; k < a1; ++k)
                r.add(OP != R_COUNT ? ldf(content, A + k) : 0.0f, !obj_mask || obj_mask[A + k] != 0,
                      static_cast<int32_t>(k - a0));
        }
        if (act) {
            if (OP == R_COUNT) {
                static_cast<int32_t *>(out)[e] = r.cnt;
            } else if (OP == R_SUM) {
                static_cast<float *>(out)[e] = r.sum;
            } else if (OP == R_PROD) {
                static_cast<float *>(out)[e] = r.prod;
            } else if (index_only) {
                static_cast<int32_t *>(out)[e] = r.bi;
            } else {
                static_cast<float *>(out)[e] = r.best;
                if (out_arg) out_arg[e] = r.bi;
            }
        }
    }
}

// Prefix offsets of the selected sub-collection without a temporary: the
// total of tile t (events [t * RB, t * RB + RB)) is staged in offsets_out at
// tile_slot(t) = min((t + 1) * RB, N), the entry whose final value is the sum
// of the counts of tiles 0..t.  An in-place inclusive scan over those entries
// makes them final; each tile then reads its exclusive prefix from the entry
// before its first event (that of tile t - 1) and writes its other entries.
__host__ __device__ inline int64_t tile_slot(int64_t t, int64_t n_events) {
    return (t + 1) * RB < n_events ? (t + 1) * RB : n_events;
}

// offsets_out[tile_slot(t)] = sum of the counts of tile t.
__global__ __launch_bounds__(RB) void tile_sums_kernel(const int32_t *counts, int64_t n_events, int64_t *offsets_out) {
    __shared__ int64_t scan_s[RB];
    const int64_t n_tiles = ceil_div(n_events, RB);
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t e = tile * RB + threadIdx.x;
        const int64_t incl = block_inclusive_scan(e < n_events ? counts[e] : 0, scan_s);
        if (threadIdx.x == RB - 1) offsets_out[tile_slot(tile, n_events)] = incl;
        __syncthreads();
    }
}

// Inclusive scan, in place, of the staged tile totals by one workgroup of
// 1024 threads (each thread a contiguous run of tiles).
__global__ __launch_bounds__(1024) void scan_tiles_kernel(int64_t *offsets_out, int64_t n_events) {
    __shared__ int64_t buf[1024];
    const int tid = threadIdx.x;
    const int64_t n = ceil_div(n_events, RB);
    const int64_t per = ceil_div(n, 1024);
    const int64_t b = tid * per;
    const int64_t e = (b + per < n) ? b + per : n;
    int64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += offsets_out[tile_slot(i, n_events)];
    buf[tid] = s;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        int64_t add = (tid >= d) ? buf[tid - d] : 0;
        __syncthreads();
        buf[tid] += add;
        __syncthreads();
    }
    int64_t run = buf[tid] - s;  // exclusive prefix of this thread's run
    for (int64_t i = b; i < e; ++i) {
        int64_t &v = offsets_out[tile_slot(i, n_events)];
        run += v;
        v = run;
    }
}

// offsets_out[0] = 0, offsets_out[e+1] = sum of counts[0..e]: the entries
// not staged (each tile's staged entry is final already and is the base the
// next tile reads, so it is not written again).
__global__ __launch_bounds__(RB) void offsets_from_counts_kernel(const int32_t *counts, int64_t n_events,
                                                                 int64_t *offsets_out) {
    __shared__ int64_t scan_s[RB];
    const int tid = threadIdx.x;
    const int64_t n_tiles = ceil_div(n_events, RB);
    if (blockIdx.x == 0 && tid == 0) offsets_out[0] = 0;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t base = tile > 0 ? offsets_out[tile * RB] : 0;
        const int64_t e = tile * RB + tid;
        const int64_t c = (e < n_events) ? counts[e] : 0;
        const int64_t incl = block_inclusive_scan(c, scan_s);
        if (e < n_events && e + 1 != tile_slot(tile, n_events)) offsets_out[e + 1] = base + incl;
        __syncthreads();
    }
}

template <typename T, int OP>
static int launch_reduce(const int64_t *off, int64_t n, const void *content, const uint8_t *om,
                         const uint8_t *em, void *out, int32_t *out_arg, int index_only, hipStream_t stream) {
    const int64_t n_wave_tiles = ceil_div(n, 64);
    const int grid = static_cast<int>(std::min<int64_t>(ceil_div(n_wave_tiles, RW), 16 * device_cus()));
    reduce_kernel<T, OP><<<grid, RB, 0, stream>>>(off, n, static_cast<const T *>(content), om, em, out,
                                                  out_arg, index_only);
    return check_launch("hepk_reduce");
}

// offsets_out from the counts just written (three launches, no temporary).
static int launch_offsets(const int32_t *counts, int64_t n, int64_t *offsets_out, hipStream_t stream) {
    const int64_t n_tiles = ceil_div(n, RB);
    const int g = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(n_tiles, 8 * device_cus())));
    if (n > 0) {
        tile_sums_kernel<<<g, RB, 0, stream>>>(counts, n, offsets_out);
        if (int rc = check_launch("hepk_reduce tile sums")) return rc;
        scan_tiles_kernel<<<1, 1024, 0, stream>>>(offsets_out, n);
        if (int rc = check_launch("hepk_reduce scan")) return rc;
    }
    offsets_from_counts_kernel<<<g, RB, 0, stream>>>(counts, n, offsets_out);
    return check_launch("hepk_reduce offsets");
}

}  // namespace hepk

extern "C" int hepk_reduce(int32_t op, const int64_t *offsets, int64_t n_events, const void *content,
                           int32_t dtype, const uint8_t *obj_mask, const uint8_t *evt_mask, void *out,
                           int32_t *out_arg, int64_t *offsets_out, hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(op >= HEPK_COUNT && op <= HEPK_PROD, "hepk_reduce: bad op %d", op);
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
    if (n_events == 0) return offsets_out ? launch_offsets(nullptr, 0, offsets_out, stream) : HEPK_OK;
    int rc;
    const bool h = dtype == HEPK_F16;
    switch (op) {
    case HEPK_COUNT:
        rc = launch_reduce<float, R_COUNT>(offsets, n_events, nullptr, obj_mask, evt_mask, out, nullptr, 0,
                                           stream);
        break;
    case HEPK_SUM:
        rc = h ? launch_reduce<_Float16, R_SUM>(offsets, n_events, content, obj_mask, evt_mask, out, nullptr, 0,
                                                stream)
               : launch_reduce<float, R_SUM>(offsets, n_events, content, obj_mask, evt_mask, out, nullptr, 0,
                                             stream);
        break;
    case HEPK_PROD:
        rc = h ? launch_reduce<_Float16, R_PROD>(offsets, n_events, content, obj_mask, evt_mask, out, nullptr, 0,
                                                 stream)
               : launch_reduce<float, R_PROD>(offsets, n_events, content, obj_mask, evt_mask, out, nullptr, 0,
                                              stream);
        break;
    case HEPK_MAX:
    case HEPK_ARGMAX:
        rc = h ? launch_reduce<_Float16, R_MAX>(offsets, n_events, content, obj_mask, evt_mask, out, out_arg,
                                                op == HEPK_ARGMAX, stream)
               : launch_reduce<float, R_MAX>(offsets, n_events, content, obj_mask, evt_mask, out, out_arg,
                                             op == HEPK_ARGMAX, stream);
        break;
    default:
        rc = h ? launch_reduce<_Float16, R_MIN>(offsets, n_events, content, obj_mask, evt_mask, out, out_arg,
                                                op == HEPK_ARGMIN, stream)
               : launch_reduce<float, R_MIN>(offsets, n_events, content, obj_mask, evt_mask, out, out_arg,
                                             op == HEPK_ARGMIN, stream);
        break;
    }
    if (rc == HEPK_OK && offsets_out)
        rc = launch_offsets(static_cast<const int32_t *>(out), n_events, offsets_out, stream);
    return rc;
}
