// hepk_match_dr: Delta-R matching of collection a against collection b in
// the same event (Sec. III: masking objects of a first collection lying
// within a Delta-R cone of an object of a second collection; Sec. IV:
// jet-lepton matching).
//
// A workgroup takes a tile of MB consecutive events.  The tile's b objects
// (a few per event) are staged once into LDS, with eta replaced by NaN for
// masked-out b so that their dR^2 is NaN and never becomes the minimum
// (exactly as skipping them).  Then one lane per a object -- coalesced reads
// of a's columns -- scans the b objects of its event in ascending order with
// a strict '<', which keeps the lowest index on ties.  Tiles whose objects
// exceed the LDS capacity fall back to one lane per event reading HBM
// directly; the arithmetic is the same.
#include "common.hpp"

namespace hepk {

constexpr int MB = 256;          // events per tile == threads per workgroup
constexpr int MACAP = 16 * MB;   // a objects per tile held in the event map
constexpr int MBCAP = 8 * MB;    // b objects per tile staged in LDS

template <typename T>
__global__ __launch_bounds__(MB) void match_dr_kernel(
    const int64_t *__restrict__ off_a, const T *__restrict__ eta_a, const T *__restrict__ phi_a,
    const uint8_t *__restrict__ mask_a, const int64_t *__restrict__ off_b, const T *__restrict__ eta_b,
    const T *__restrict__ phi_b, const uint8_t *__restrict__ mask_b, int64_t n_events, float thr2,
    float *__restrict__ min_dr2, int32_t *__restrict__ idx_b, uint8_t *__restrict__ clean) {
    __shared__ int32_t offa_s[MB + 1], offb_s[MB + 1];
    __shared__ float beta_s[MBCAP], bphi_s[MBCAP];
    __shared__ uint16_t aev_s[MACAP];
    const int tid = threadIdx.x;
    const int64_t n_tiles = ceil_div(n_events, MB);
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t e0 = tile * MB;
        const int ne = static_cast<int>(n_events - e0 < MB ? n_events - e0 : MB);
        const int64_t A0 = off_a[e0], A1 = off_a[e0 + ne];
        const int64_t B0 = off_b[e0], B1 = off_b[e0 + ne];
        if (A1 - A0 > MACAP || B1 - B0 > MBCAP) {
            // direct path: one lane per event, everything from HBM
            if (tid < ne) {
                const int64_t e = e0 + tid;
                const int64_t b0 = off_b[e], b1 = off_b[e + 1];
                for (int64_t a = off_a[e]; a < off_a[e + 1]; ++a) {
                    const float ea = ldf(eta_a, a), pa = ldf(phi_a, a);
                    float best = INFINITY;
                    int32_t bi = -1;
                    for (int64_t b = b0; b < b1; ++b) {
                        if (mask_b && !mask_b[b]) continue;
                        const float d2 = delta_r2(ea, pa, ldf(eta_b, b), ldf(phi_b, b));
                        if (d2 < best) {
                            best = d2;
                            bi = static_cast<int32_t>(b - b0);
                        }
                    }
                    if (min_dr2) min_dr2[a] = best;
                    if (idx_b) idx_b[a] = bi;
                    if (clean) clean[a] = ((!mask_a || mask_a[a]) && !(best <= thr2)) ? 1 : 0;
                }
            }
            continue;
        }
        const int na = static_cast<int>(A1 - A0), nb = static_cast<int>(B1 - B0);
        if (tid < ne) {
            offa_s[tid] = static_cast<int32_t>(off_a[e0 + tid] - A0);
            offb_s[tid] = static_cast<int32_t>(off_b[e0 + tid] - B0);
        }
        if (tid == 0) {
            offa_s[ne] = na;
            offb_s[ne] = nb;
        }
        for (int b = tid; b < nb; b += MB) {
            float e = ldf(eta_b, B0 + b);
            if (mask_b && !mask_b[B0 + b]) e = __builtin_nanf("");
            beta_s[b] = e;
            bphi_s[b] = ldf(phi_b, B0 + b);
        }
        __syncthreads();
        if (tid < ne)
            for (int k = offa_s[tid]; k < offa_s[tid + 1]; ++k) aev_s[k] = static_cast<uint16_t>(tid);
        __syncthreads();
        for (int a = tid; a < na; a += MB) {
            const int ev = aev_s[a];
            const float ea = ldf(eta_a, A0 + a), pa = ldf(phi_a, A0 + a);
            const int b0 = offb_s[ev], b1 = offb_s[ev + 1];
            float best = INFINITY;
            int32_t bi = -1;
            for (int b = b0; b < b1; ++b) {
                const float d2 = delta_r2(ea, pa, beta_s[b], bphi_s[b]);
                if (d2 < best) {
                    best = d2;
                    bi = b - b0;
                }
            }
            if (min_dr2) min_dr2[A0 + a] = best;
            if (idx_b) idx_b[A0 + a] = bi;
            if (clean) clean[A0 + a] = ((!mask_a || mask_a[A0 + a]) && !(best <= thr2)) ? 1 : 0;
        }
        __syncthreads();
    }
}

}  // namespace hepk

extern "C" int hepk_match_dr(const int64_t *off_a, const void *eta_a, const void *phi_a, const uint8_t *mask_a,
                             const int64_t *off_b, const void *eta_b, const void *phi_b, const uint8_t *mask_b,
                             int32_t dtype, int64_t n_events, float dr, float *min_dr2, int32_t *idx_b,
                             uint8_t *clean_out, hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(n_events >= 0, "hepk_match_dr: n_events < 0");
    HEPK_REQUIRE(off_a && off_b, "hepk_match_dr: offsets are NULL");
    HEPK_REQUIRE(eta_a && phi_a && eta_b && phi_b, "hepk_match_dr: eta/phi column is NULL");
    if (dtype != HEPK_F32 && dtype != HEPK_F16) {
        set_error("hepk_match_dr: dtype %d unsupported", dtype);
        return HEPK_EUNSUPPORTED;
    }
    if (n_events == 0 || (!min_dr2 && !idx_b && !clean_out)) return HEPK_OK;
    const float thr2 = dr * dr;  // rounded once to float32
    const int64_t n_tiles = ceil_div(n_events, MB);
    const int grid = static_cast<int>(std::min<int64_t>(n_tiles, 8 * device_cus()));
    if (dtype == HEPK_F16)
        match_dr_kernel<_Float16><<<grid, MB, 0, stream>>>(
            off_a, static_cast<const _Float16 *>(eta_a), static_cast<const _Float16 *>(phi_a), mask_a, off_b,
            static_cast<const _Float16 *>(eta_b), static_cast<const _Float16 *>(phi_b), mask_b, n_events, thr2,
            min_dr2, idx_b, clean_out);
    else
        match_dr_kernel<float><<<grid, MB, 0, stream>>>(
            off_a, static_cast<const float *>(eta_a), static_cast<const float *>(phi_a), mask_a, off_b,
            static_cast<const float *>(eta_b), static_cast<const float *>(phi_b), mask_b, n_events, thr2,
            min_dr2, idx_b, clean_out);
    return check_launch("hepk_match_dr");
}
