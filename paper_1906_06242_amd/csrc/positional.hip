// Positional kernels over jagged collections (Sec. III): get_in_offsets and
// set_in_offsets retrieve or set the n-th selected element of every event,
// select_opposite_sign_muons keeps per event the first two objects in pT
// order with opposite charges, and compaction gathers the selected objects
// into a contiguous collection laid out by the offsets of their counts.
//
// get/set and the opposite-sign selection touch a few bytes per event: one
// lane per event walks its objects (consecutive lanes read consecutive
// events' bytes, so the loads of a wavefront share cache lines).
// Compaction moves every selected element: each wavefront owns tiles of 64
// consecutive events, takes their objects 64 at a time in order, and places
// the kept ones by a wavefront ballot and prefix count, so both its reads and
// its writes are contiguous runs.
#include "common.hpp"

namespace hepk {

// Workgroups per CU, at most: a sweep of 8-64 put the best at 64 (get/set 7%,
// opposite-sign pairs 4% faster than 16).
constexpr int kTileWgPerCu = 64;

constexpr int PB = 256;

// Content index of the n-th (from 0) object of [i0, i1) with m set (every
// object when m is NULL); -1 when there are fewer.
// The first kNthBatch mask bytes are read in one batch (indices clamped
// into the range, so no read waits on another); only a range whose n-th
// selected object lies beyond them goes on byte by byte.
constexpr int kNthBatch = 8;
__device__ __forceinline__ int64_t nth_selected(int64_t i0, int64_t i1, const uint8_t *m, int32_t n) {
    if (n < 0) return -1;
    if (!m) return (n < i1 - i0) ? i0 + n : -1;
    const int64_t len = i1 - i0;
    if (len <= 0) return -1;
    uint32_t b[kNthBatch];
#pragma unroll
    for (int k = 0; k < kNthBatch; ++k) b[k] = m[i0 + min<int64_t>(k, len - 1)];
    int32_t seen = 0;
    int64_t found = -1;
#pragma unroll
    for (int k = 0; k < kNthBatch; ++k) {
        const bool hit = k < len && b[k] != 0u;
        found = (hit && seen == n && found < 0) ? i0 + k : found;
        seen += hit ? 1 : 0;
    }
    if (found >= 0 || len <= kNthBatch) return found;
    for (int64_t i = i0 + kNthBatch; i < i1; ++i) {
        if (!m[i]) continue;
        if (seen == n) return i;
        ++seen;
    }
    return -1;
}

template <typename T>
__global__ __launch_bounds__(PB) void get_in_offsets_kernel(const int64_t *__restrict__ off, int64_t n_events,
                                                            const T *__restrict__ content,
                                                            const uint8_t *__restrict__ om,
                                                            const uint8_t *__restrict__ em,
                                                            const int32_t *__restrict__ idx, int32_t n, float fill,
                                                            float *__restrict__ out, int32_t *__restrict__ out_index) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * PB;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * PB + threadIdx.x; e < n_events; e += stride) {
        const int64_t i0 = off[e], i1 = off[e + 1];
        int64_t i = -1;
        if (!em || em[e]) i = nth_selected(i0, i1, om, idx ? idx[e] : n);
        out[e] = i >= 0 ? ldf(content, i) : fill;
        if (out_index) out_index[e] = i >= 0 ? static_cast<int32_t>(i - i0) : -1;
    }
}

template <typename T>
__global__ __launch_bounds__(PB) void set_in_offsets_kernel(const int64_t *__restrict__ off, int64_t n_events,
                                                            T *__restrict__ content, const uint8_t *__restrict__ om,
                                                            const uint8_t *__restrict__ em,
                                                            const int32_t *__restrict__ idx, int32_t n, T value) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * PB;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * PB + threadIdx.x; e < n_events; e += stride) {
        if (em && !em[e]) continue;
        const int64_t i = nth_selected(off[e], off[e + 1], om, idx ? idx[e] : n);
        if (i >= 0) content[i] = value;
    }
}

// i comes before j in pT order: larger pt first, NaN after every number,
// equal (or both NaN) pt by lower index.
__device__ __forceinline__ bool pt_before(float pi, int64_t i, float pj, int64_t j) {
    const bool ni = pi != pi, nj = pj != pj;
    if (ni != nj) return nj;
    if (!ni && pi != pj) return pi > pj;
    return i < j;
}

__device__ __forceinline__ bool opposite_sign(int32_t a, int32_t b) { return (a > 0 && b < 0) || (a < 0 && b > 0); }

// Per event, the first pair (p, r), p before r in pT order, of selected
// objects with charges of opposite sign -- which is always the highest-pT
// object of positive charge and the highest-pT object of negative charge:
// with both present, say the positive one P first, every selected object
// before P has charge 0 (P is the first positive and the first negative
// comes after it), so P is the first object with a partner after it and
// its first partner is the first negative; with either absent there is no
// pair.  So one pass keeps the best (in pT order) positive and negative
// object.  Both get mask 1, every other object of the event 0.  Events of
// up to kOsRegs objects are read into registers in one batch (indices
// clamped into the event, so no load waits on another); larger ones are
// scanned straight from memory.
constexpr int kOsRegs = 8;

template <typename T>
__global__ __launch_bounds__(PB) void opposite_sign_kernel(const int64_t *__restrict__ off, int64_t n_events,
                                                           const T *__restrict__ pt, const int32_t *__restrict__ q,
                                                           const uint8_t *__restrict__ om,
                                                           uint8_t *__restrict__ out) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * PB;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * PB + threadIdx.x; e < n_events; e += stride) {
        const int64_t i0 = off[e], i1 = off[e + 1];
        const int64_t n = i1 - i0;
        // best positive and negative object so far (local index, its pt)
        int64_t bp = -1, bn = -1;
        float pp = 0.0f, pn = 0.0f;
        auto take = [&](bool sel, int32_t c, float pa, int64_t a) {
            if (sel && c > 0 && (bp < 0 || pt_before(pa, a, pp, bp))) {
                bp = a;
                pp = pa;
            }
            if (sel && c < 0 && (bn < 0 || pt_before(pa, a, pn, bn))) {
                bn = a;
                pn = pa;
            }
        };
        if (n <= kOsRegs) {
            float p[kOsRegs];
            int32_t c[kOsRegs];
            uint32_t m[kOsRegs];
#pragma unroll
            for (int k = 0; k < kOsRegs; ++k) {
                p[k] = 0.0f;
                c[k] = 0;
                m[k] = 0u;
            }
            if (n > 0) {
#pragma unroll
                for (int k = 0; k < kOsRegs; ++k) {
                    const int64_t ix = i0 + min<int64_t>(k, n - 1);
                    p[k] = ldf(pt, ix);
                    c[k] = q[ix];
                    m[k] = om ? static_cast<uint32_t>(om[ix]) : 1u;
                }
            }
#pragma unroll
            for (int k = 0; k < kOsRegs; ++k) take((k < n) & (m[k] != 0u), c[k], p[k], k);
            const bool pair = bp >= 0 && bn >= 0;
#pragma unroll
            for (int k = 0; k < kOsRegs; ++k)
                if (k < n) out[i0 + k] = (pair && (k == bp || k == bn)) ? 1 : 0;
            continue;
        }
        for (int64_t a = 0; a < n; ++a) {
            out[i0 + a] = 0;
            take(!om || om[i0 + a] != 0, q[i0 + a], ldf(pt, i0 + a), a);
        }
        if (bp >= 0 && bn >= 0) {
            out[i0 + bp] = 1;
            out[i0 + bn] = 1;
        }
    }
}

// Compaction: each wavefront a tile of 64 events; the tile's objects 64 at a
// time, kept ones placed at base + (kept objects of the tile before them),
// base = offsets_out[first event of the tile].  ES: element size in bytes.
template <int ES>
struct Elem;
template <>
struct Elem<1> {
    using T = uint8_t;
};
template <>
struct Elem<2> {
    using T = uint16_t;
};
template <>
struct Elem<4> {
    using T = uint32_t;
};

constexpr int kCompactChunks = 8;  // chunks of 64 objects a tile reads in one batch

template <int ES>
__global__ __launch_bounds__(PB) void compact_kernel(const int64_t *__restrict__ off, int64_t n_events,
                                                     const typename Elem<ES>::T *__restrict__ content,
                                                     const uint8_t *__restrict__ om,
                                                     const int64_t *__restrict__ offsets_out, int64_t n_out,
                                                     typename Elem<ES>::T *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = static_cast<int64_t>(blockIdx.x) * (PB / 64) + (threadIdx.x >> 6);
    const int64_t n_waves = static_cast<int64_t>(gridDim.x) * (PB / 64);
    const int64_t n_tiles = ceil_div(n_events, 64);
    for (int64_t t = wave; t < n_tiles; t += n_waves) {
        const int64_t e0 = t * 64;
        const int64_t e1 = min<int64_t>(e0 + 64, n_events);
        const int64_t A = as_const(off)[e0], B = as_const(off)[e1];
        int64_t base = as_const(offsets_out)[e0];
        if (B - A <= 64 * kCompactChunks) {
            // the whole tile: every chunk's mask bytes and elements as
            // buffer loads over exactly [A, B) (0 past the end), all in
            // flight and waited for once
            const int nobj = static_cast<int>(B - A);
            const buf_t bc = buf_span(content + A, static_cast<uint32_t>(nobj) * ES);
            const buf_t bm = buf_span(om ? static_cast<const void *>(om + A) : static_cast<const void *>(content),
                                      om ? static_cast<uint32_t>(nobj) : 0u);
            uint32_t mk[kCompactChunks], v[kCompactChunks];
#pragma unroll
            for (int c = 0; c < kCompactChunks; ++c) {
                const int i = lane + 64 * c;
                mk[c] = om ? __builtin_amdgcn_raw_buffer_load_b8(bm, i, 0, kBufNt) : 1u;
                if constexpr (ES == 4)
                    v[c] = __builtin_amdgcn_raw_buffer_load_b32(bc, i * 4, 0, kBufNt);
                else if constexpr (ES == 2)
                    v[c] = __builtin_amdgcn_raw_buffer_load_b16(bc, i * 2, 0, kBufNt);
                else
                    v[c] = __builtin_amdgcn_raw_buffer_load_b8(bc, i, 0, kBufNt);
            }
#pragma unroll
            for (int c = 0; c < kCompactChunks; ++c) asm volatile("" ::"v"(mk[c]), "v"(v[c]));
#pragma unroll
            for (int c = 0; c < kCompactChunks; ++c) {
                if (64 * c >= nobj) break;
                const bool keep = (lane + 64 * c < nobj) & (mk[c] != 0u);
                const uint64_t bal = __ballot(keep);
                const int before = static_cast<int>(__builtin_amdgcn_mbcnt_hi(
                    static_cast<uint32_t>(bal >> 32), __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(bal), 0u)));
                const int64_t dst = base + before;
                if (keep && dst < n_out) out[dst] = static_cast<typename Elem<ES>::T>(v[c]);
                base += __popcll(bal);
            }
            continue;
        }
        for (int64_t k0 = A; k0 < B; k0 += 64) {
            const int64_t i = k0 + lane;
            const bool in = i < B;
            const bool keep = in && (!om || om[i] != 0);
            typename Elem<ES>::T v{};
            if (keep) v = content[i];
            const uint64_t bal = __ballot(keep);
            const int before = static_cast<int>(__builtin_amdgcn_mbcnt_hi(
                static_cast<uint32_t>(bal >> 32), __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(bal), 0u)));
            const int64_t dst = base + before;
            if (keep && dst < n_out) out[dst] = v;
            base += __popcll(bal);
        }
    }
}

static int grid_for(int64_t rows, int per_thread = 1) {
    return static_cast<int>(
        std::max<int64_t>(1, std::min<int64_t>(ceil_div(ceil_div(rows, per_thread), PB), kTileWgPerCu * device_cus())));
}

}  // namespace hepk

extern "C" int hepk_get_in_offsets(const int64_t *offsets, int64_t n_events, const void *content, int32_t dtype,
                                   const uint8_t *obj_mask, const uint8_t *evt_mask, const int32_t *idx, int32_t n,
                                   float fill, float *out, int32_t *out_index, hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(n_events >= 0 && offsets, "hepk_get_in_offsets: bad offsets or n_events");
    HEPK_REQUIRE(n_events == 0 || (content && out), "hepk_get_in_offsets: content or out is NULL");
    HEPK_REQUIRE(dtype == HEPK_F32 || dtype == HEPK_F16, "hepk_get_in_offsets: dtype %d not F32 or F16", dtype);
    if (n_events == 0) return HEPK_OK;
    const int g = grid_for(n_events);
    if (dtype == HEPK_F16)
        get_in_offsets_kernel<_Float16><<<g, PB, 0, stream>>>(offsets, n_events, static_cast<const _Float16 *>(content),
                                                               obj_mask, evt_mask, idx, n, fill, out, out_index);
    else
        get_in_offsets_kernel<float><<<g, PB, 0, stream>>>(offsets, n_events, static_cast<const float *>(content),
                                                            obj_mask, evt_mask, idx, n, fill, out, out_index);
    return check_launch("hepk_get_in_offsets");
}

extern "C" int hepk_set_in_offsets(const int64_t *offsets, int64_t n_events, void *content, int32_t dtype,
                                   const uint8_t *obj_mask, const uint8_t *evt_mask, const int32_t *idx, int32_t n,
                                   float value, hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(n_events >= 0 && offsets, "hepk_set_in_offsets: bad offsets or n_events");
    HEPK_REQUIRE(n_events == 0 || content, "hepk_set_in_offsets: content is NULL");
    HEPK_REQUIRE(dtype == HEPK_F32 || dtype == HEPK_U8, "hepk_set_in_offsets: dtype %d not F32 or U8", dtype);
    if (n_events == 0) return HEPK_OK;
    const int g = grid_for(n_events);
    if (dtype == HEPK_U8)
        set_in_offsets_kernel<uint8_t><<<g, PB, 0, stream>>>(offsets, n_events, static_cast<uint8_t *>(content),
                                                              obj_mask, evt_mask, idx, n,
                                                              static_cast<uint8_t>(value != 0.0f ? 1 : 0));
    else
        set_in_offsets_kernel<float><<<g, PB, 0, stream>>>(offsets, n_events, static_cast<float *>(content), obj_mask,
                                                            evt_mask, idx, n, value);
    return check_launch("hepk_set_in_offsets");
}

extern "C" int hepk_select_opposite_sign(const int64_t *offsets, int64_t n_events, const void *pt, int32_t dtype,
                                         const int32_t *charge, const uint8_t *obj_mask, uint8_t *mask_out,
                                         hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(n_events >= 0 && offsets, "hepk_select_opposite_sign: bad offsets or n_events");
    HEPK_REQUIRE(n_events == 0 || (pt && charge && mask_out), "hepk_select_opposite_sign: NULL column or output");
    HEPK_REQUIRE(dtype == HEPK_F32 || dtype == HEPK_F16, "hepk_select_opposite_sign: dtype %d not F32 or F16", dtype);
    if (n_events == 0) return HEPK_OK;
    const int g = grid_for(n_events);
    if (dtype == HEPK_F16)
        opposite_sign_kernel<_Float16><<<g, PB, 0, stream>>>(offsets, n_events, static_cast<const _Float16 *>(pt),
                                                              charge, obj_mask, mask_out);
    else
        opposite_sign_kernel<float><<<g, PB, 0, stream>>>(offsets, n_events, static_cast<const float *>(pt), charge,
                                                           obj_mask, mask_out);
    return check_launch("hepk_select_opposite_sign");
}

extern "C" int hepk_compact(const int64_t *offsets, int64_t n_events, const void *content, int32_t dtype,
                            const uint8_t *obj_mask, const int64_t *offsets_out, int64_t n_out, void *out,
                            hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(n_events >= 0 && offsets && offsets_out, "hepk_compact: bad offsets or n_events");
    HEPK_REQUIRE(n_out >= 0 && (n_out == 0 || out), "hepk_compact: bad output");
    HEPK_REQUIRE(n_events == 0 || content, "hepk_compact: content is NULL");
    HEPK_REQUIRE(dtype >= HEPK_F32 && dtype <= HEPK_U8, "hepk_compact: bad dtype %d", dtype);
    if (n_events == 0 || n_out == 0) return HEPK_OK;
    const int g = static_cast<int>(
        std::max<int64_t>(1, std::min<int64_t>(ceil_div(ceil_div(n_events, 64), PB / 64), kTileWgPerCu * device_cus())));
    if (dtype == HEPK_U8)
        compact_kernel<1><<<g, PB, 0, stream>>>(offsets, n_events, static_cast<const uint8_t *>(content), obj_mask,
                                                offsets_out, n_out, static_cast<uint8_t *>(out));
    else if (dtype == HEPK_F16)
        compact_kernel<2><<<g, PB, 0, stream>>>(offsets, n_events, static_cast<const uint16_t *>(content), obj_mask,
                                                offsets_out, n_out, static_cast<uint16_t *>(out));
    else
        compact_kernel<4><<<g, PB, 0, stream>>>(offsets, n_events, static_cast<const uint32_t *>(content), obj_mask,
                                                offsets_out, n_out, static_cast<uint32_t *>(out));
    return check_launch("hepk_compact");
}
