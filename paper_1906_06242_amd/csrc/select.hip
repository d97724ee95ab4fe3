// hepk_select: AND of up to HEPK_MAX_CUTS column cuts into a byte mask
// (Sec. III object/event masks; Sec. IV object selection on pt and eta,
// event selection on event variables).
//
// Elementwise and HBM-bound: a thread takes groups of 4 consecutive rows,
// reads each from every cut's column with one 16-byte (float32, int32) or
// 8-byte (float16) nontemporal load -- all loads of a step issued before any
// compare, the cut count a template parameter so no loop over cuts remains
// -- and writes the 4 mask bytes as one 32-bit store.
#include "common.hpp"

namespace hepk {

struct CutDev {
    const void *col;
    int32_t dtype;
    int32_t op;
    float thr;
    int32_t ithr;
};

struct SelectArgs {
    CutDev cut[HEPK_MAX_CUTS];
    int32_t n_cuts;
};

__device__ __forceinline__ bool row_passes(const SelectArgs &a, int64_t i) {
    bool ok = true;
    for (int k = 0; k < a.n_cuts; ++k) {
        const CutDev &c = a.cut[k];
        bool p;
        if (c.dtype == HEPK_I32)
            p = cmp_i(static_cast<const int32_t *>(c.col)[i], c.op, c.ithr);
        else if (c.dtype == HEPK_F16)
            p = cmp_f(ldf(static_cast<const _Float16 *>(c.col), i), c.op, c.thr);
        else
            p = cmp_f(ldf(static_cast<const float *>(c.col), i), c.op, c.thr);
        ok = ok && p;
    }
    return ok;
}

// Rows [0, n) in groups of four (mask_in/mask_out 4-byte aligned, columns
// 16-byte (float32, int32) or 8-byte (float16) aligned), NC cuts known at
// compile time; the last, partial group row by row with byte stores.  Each
// thread takes U groups per step, spaced a grid apart, and issues every load
// of the step (U groups x NC columns + the mask words) before the first
// compare; indices past the end are clamped onto the last group so that no
// load needs a branch, and only groups in range are stored.  Every byte is
// read and written once, so loads and stores are nontemporal.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Groups per thread per step: two for a single column, else one (a sweep of
// 1-8 loads in flight per thread and 2-64 workgroups per CU on 1e7-1e8 rows
// put the best at 1-2 loads and up to 64 workgroups per CU).
template <int NC>
constexpr int sel_groups() {
    return NC <= 1 ? 2 : 1;
}
constexpr int kSelWgPerCu = 64;

template <int NC, int U>
__global__ __launch_bounds__(256) void select_vec4_kernel(SelectArgs a, int64_t n, const uint32_t *mask_in,
                                                          uint32_t *mask_out) {
    const int64_t n4 = n / 4;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (gid == 0 && 4 * n4 < n) {
        const uint8_t *mi = reinterpret_cast<const uint8_t *>(mask_in);
        uint8_t *mo = reinterpret_cast<uint8_t *>(mask_out);
        for (int64_t i = 4 * n4; i < n; ++i) mo[i] = ((!mi || mi[i] != 0) && row_passes(a, i)) ? 1 : 0;
    }
    for (int64_t g0 = gid; g0 < n4; g0 += U * stride) {
        u32x4 raw[U][NC > 0 ? NC : 1];
        uint32_t m[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t g = g0 + u * stride < n4 ? g0 + u * stride : n4 - 1;
#pragma unroll
            for (int k = 0; k < NC; ++k) {
                const CutDev &c = a.cut[k];
                if (c.dtype == HEPK_F16) {
                    const u32x2 h = __builtin_nontemporal_load(static_cast<const u32x2 *>(c.col) + g);
                    raw[u][k] = u32x4{h.x, h.y, 0u, 0u};
                } else {
                    raw[u][k] = __builtin_nontemporal_load(static_cast<const u32x4 *>(c.col) + g);
                }
            }
            m[u] = mask_in ? __builtin_nontemporal_load(mask_in + g) : 0x01010101u;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            uint32_t out = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                bool p = ((m[u] >> (8 * r)) & 0xffu) != 0;
#pragma unroll
                for (int k = 0; k < NC; ++k) {
                    const CutDev &c = a.cut[k];
                    const uint32_t w[4] = {raw[u][k].x, raw[u][k].y, raw[u][k].z, raw[u][k].w};
                    bool q;
                    if (c.dtype == HEPK_I32) {
                        q = cmp_i(static_cast<int32_t>(w[r]), c.op, c.ithr);
                    } else if (c.dtype == HEPK_F16) {
                        const uint16_t bits16 = static_cast<uint16_t>(w[r >> 1] >> (16 * (r & 1)));
                        q = cmp_f(static_cast<float>(__builtin_bit_cast(_Float16, bits16)), c.op, c.thr);
                    } else {
                        q = cmp_f(__builtin_bit_cast(float, w[r]), c.op, c.thr);
                    }
                    p = p && q;
                }
                out |= (p ? 1u : 0u) << (8 * r);
            }
            if (g0 + u * stride < n4) __builtin_nontemporal_store(out, mask_out + g0 + u * stride);
        }
    }
}

template <int NC>
static void launch_vec4(const SelectArgs &a, int64_t n, const uint32_t *mask_in, uint32_t *mask_out,
                        hipStream_t stream) {
    constexpr int U = sel_groups<NC>();
    const int64_t per_wg = 256 * static_cast<int64_t>(U);
    const int64_t want = std::max<int64_t>(1, ceil_div(n / 4, per_wg));
    const int grid = static_cast<int>(std::min<int64_t>(want, kSelWgPerCu * device_cus()));
    select_vec4_kernel<NC, U><<<grid, 256, 0, stream>>>(a, n, mask_in, mask_out);
}

// Rows [begin, n) one per thread (unaligned masks or columns).
__global__ void select_scalar_kernel(SelectArgs a, int64_t begin, int64_t n, const uint8_t *mask_in,
                                     uint8_t *mask_out) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t i = begin + static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        bool in = mask_in ? (mask_in[i] != 0) : true;
        mask_out[i] = (in && row_passes(a, i)) ? 1 : 0;
    }
}

}  // namespace hepk

extern "C" int hepk_select(const hepk_cut *cuts, int32_t n_cuts, int64_t n, const uint8_t *mask_in,
                           uint8_t *mask_out, hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(n >= 0, "hepk_select: n < 0");
    HEPK_REQUIRE(n_cuts >= 0 && n_cuts <= HEPK_MAX_CUTS, "hepk_select: n_cuts %d not in [0, %d]",
                 n_cuts, HEPK_MAX_CUTS);
    HEPK_REQUIRE(n_cuts == 0 || cuts, "hepk_select: cuts is NULL");
    HEPK_REQUIRE(n == 0 || mask_out, "hepk_select: mask_out is NULL");
    SelectArgs a{};
    a.n_cuts = n_cuts;
    for (int k = 0; k < n_cuts; ++k) {
        HEPK_REQUIRE(cuts[k].dtype == HEPK_F32 || cuts[k].dtype == HEPK_F16 || cuts[k].dtype == HEPK_I32,
                     "hepk_select: cut %d has bad dtype %d", k, cuts[k].dtype);
        HEPK_REQUIRE(cuts[k].op >= HEPK_GT && cuts[k].op <= HEPK_ABS_LE, "hepk_select: cut %d has bad op %d",
                     k, cuts[k].op);
        HEPK_REQUIRE(n == 0 || cuts[k].col, "hepk_select: cut %d column is NULL", k);
        a.cut[k] = CutDev{cuts[k].col, cuts[k].dtype, cuts[k].op, cuts[k].thr, cuts[k].ithr};
    }
    if (n == 0) return HEPK_OK;
    const int block = 256;
    const int max_grid = 64 * device_cus();
    bool aligned = (reinterpret_cast<uintptr_t>(mask_out) % 4 == 0) &&
                   (!mask_in || reinterpret_cast<uintptr_t>(mask_in) % 4 == 0);
    for (int k = 0; k < n_cuts; ++k)
        aligned = aligned && reinterpret_cast<uintptr_t>(cuts[k].col) % (cuts[k].dtype == HEPK_F16 ? 8 : 16) == 0;
    if (aligned) {
        const uint32_t *mi = reinterpret_cast<const uint32_t *>(mask_in);
        uint32_t *mo = reinterpret_cast<uint32_t *>(mask_out);
        static_assert(HEPK_MAX_CUTS == 8, "one case per cut count");
        switch (n_cuts) {
            case 0: launch_vec4<0>(a, n, mi, mo, stream); break;
            case 1: launch_vec4<1>(a, n, mi, mo, stream); break;
            case 2: launch_vec4<2>(a, n, mi, mo, stream); break;
            case 3: launch_vec4<3>(a, n, mi, mo, stream); break;
            case 4: launch_vec4<4>(a, n, mi, mo, stream); break;
            case 5: launch_vec4<5>(a, n, mi, mo, stream); break;
            case 6: launch_vec4<6>(a, n, mi, mo, stream); break;
            case 7: launch_vec4<7>(a, n, mi, mo, stream); break;
            default: launch_vec4<8>(a, n, mi, mo, stream); break;
        }
        return check_launch("hepk_select");
    }
    const int grid = static_cast<int>(std::min<int64_t>(ceil_div(n, block), max_grid));
    select_scalar_kernel<<<grid, block, 0, stream>>>(a, 0, n, mask_in, mask_out);
    return check_launch("hepk_select");
}
