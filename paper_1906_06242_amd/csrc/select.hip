// hepk_select: AND of up to HEPK_MAX_CUTS column cuts into a byte mask
// (Sec. III object/event masks; Sec. IV object selection on pt and eta,
// event selection on event variables).
//
// Elementwise and HBM-bound: each thread owns 4 consecutive rows, so the
// mask is written as one 32-bit store per thread and every column read is a
// fully used 1 KiB span per wavefront instruction.
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

// Rows [0, 4*n4) in groups of four; mask_in/mask_out 4-byte aligned.
__global__ void select_vec4_kernel(SelectArgs a, int64_t n4, const uint32_t *mask_in, uint32_t *mask_out) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * blockDim.x;
    for (int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; g < n4; g += stride) {
        uint32_t m = mask_in ? mask_in[g] : 0x01010101u;
        uint32_t out = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            bool in = ((m >> (8 * k)) & 0xffu) != 0;
            bool p = in && row_passes(a, 4 * g + k);
            out |= (p ? 1u : 0u) << (8 * k);
        }
        mask_out[g] = out;
    }
}

// Rows [begin, n) one per thread (tails and unaligned masks).
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
    const int max_grid = 8 * device_cus();
    const bool aligned = (reinterpret_cast<uintptr_t>(mask_out) % 4 == 0) &&
                         (!mask_in || reinterpret_cast<uintptr_t>(mask_in) % 4 == 0);
    int64_t done = 0;
    if (aligned && n >= 4) {
        const int64_t n4 = n / 4;
        int grid = static_cast<int>(std::min<int64_t>(ceil_div(n4, block), max_grid));
        select_vec4_kernel<<<grid, block, 0, stream>>>(a, n4, reinterpret_cast<const uint32_t *>(mask_in),
                                                       reinterpret_cast<uint32_t *>(mask_out));
        int rc = check_launch("hepk_select");
        if (rc) return rc;
        done = 4 * n4;
    }
    if (done < n) {
        int grid = static_cast<int>(std::min<int64_t>(ceil_div(n - done, block), max_grid));
        select_scalar_kernel<<<grid, block, 0, stream>>>(a, done, n, mask_in, mask_out);
        return check_launch("hepk_select");
    }
    return HEPK_OK;
}
