// hepk_match_dr: Delta-R matching of collection a against collection b in
// the same event (Sec. III: masking objects of a first collection lying
// within a Delta-R cone of an object of a second collection; Sec. IV:
// jet-lepton matching).
//
// Each wavefront owns tiles of 64 consecutive events and works through them
// without waiting for the rest of its workgroup.  For one tile it reads the
// two object ranges with scalar loads, then issues every load of the tile at
// once: both offsets of each event lane's event in a and b, up to MKA a
// objects and MKB b objects per lane (consecutive lanes, consecutive
// objects).  The b objects go to the wavefront's LDS with eta replaced by NaN
// for masked-out b, so that their dR^2 is NaN and never becomes the minimum
// (exactly as skipping them); each event lane writes its event's b range over
// its a objects; then each a lane scans the b objects of its event in
// ascending order with a strict '<', which keeps the lowest index on ties.
// Tiles whose objects exceed the register capacity fall back to one lane per
// event reading HBM directly; the arithmetic is the same.
#include "common.hpp"

namespace hepk {

// Workgroups per CU, at most: a sweep of 8-64 put the best at 64 (16: 5% slower).
constexpr int kTileWgPerCu = 64;

constexpr int MW = 4;    // wavefronts per workgroup
constexpr int MKA = 8;   // a objects per lane: 512 per tile
constexpr int MKB = 4;   // b objects per lane: 256 per tile

__device__ __forceinline__ void wave_fence_dr() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Mask bytes of a tile are read as the aligned 4-byte words that hold them
// (one load moves four masks; every word holds a byte of the range, so it
// lies in the buffer's pages): mask_words issues the loads, mask_stage puts
// them into the wavefront's LDS and returns where byte 0 of the range is.
constexpr int MBW = (64 * MKB + 3 + 255) / 256;  // mask words per lane, b objects
constexpr int MAW = (64 * MKA + 3 + 255) / 256;  // and a objects
template <int W>
struct MaskWords {
    uint32_t v[W];
    int s, nw;
};
template <int W>
__device__ __forceinline__ MaskWords<W> mask_words(const uint8_t *p, int n, int lane) {
    MaskWords<W> m;
    m.s = static_cast<int>(reinterpret_cast<uintptr_t>(p) & 3u);
    m.nw = n > 0 ? (n + m.s + 3) >> 2 : 0;
    // buffer loads over exactly the nw words (0 past them): no branch per word
    const buf_t bw = buf_span(p - m.s, static_cast<uint32_t>(m.nw) * 4u);
#pragma unroll
    for (int k = 0; k < W; ++k) m.v[k] = buf_u32(bw, (lane + 64 * k) * 4);
    return m;
}
template <int W>
__device__ __forceinline__ const uint8_t *mask_stage(const MaskWords<W> &m, uint32_t *lds, int lane) {
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const int w = lane + 64 * k;
        if (w < m.nw) lds[w] = m.v[k];
    }
    return reinterpret_cast<const uint8_t *>(lds) + m.s;
}

template <typename T>
__global__ __launch_bounds__(64 * MW) void match_dr_kernel(
    const int64_t *__restrict__ off_a, const T *__restrict__ eta_a, const T *__restrict__ phi_a,
    const uint8_t *__restrict__ mask_a, const int64_t *__restrict__ off_b, const T *__restrict__ eta_b,
    const T *__restrict__ phi_b, const uint8_t *__restrict__ mask_b, int64_t n_events, float thr2,
    float *__restrict__ min_dr2, int32_t *__restrict__ idx_b, uint8_t *__restrict__ clean) {
    static_assert(__is_same(T, float) || __is_same(T, _Float16), "content is float32 or float16 (raw_f)");
    __shared__ float beta_s[MW][64 * MKB + 2], bphi_s[MW][64 * MKB + 2];  // +2: reads past a range's end
    __shared__ uint32_t arng_s[MW][64 * MKA];  // per a object: its event's b range (first | count << 16)
    __shared__ uint32_t mskb_s[MW][64 * MBW], mska_s[MW][64 * MAW];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    float *be = beta_s[wave], *bp = bphi_s[wave];
    uint32_t *ar = arng_s[wave];
    const int64_t n_tiles = ceil_div(n_events, 64);
    const int64_t step = static_cast<int64_t>(gridDim.x) * MW;
    // the object ranges of a tile are fetched one tile ahead (scalar loads
    // that overlap the current tile's work)
    int64_t nb4[4] = {0, 0, 0, 0};
    auto bounds = [&](int64_t t) {
        const int64_t e0 = t * 64, e1 = e0 + min<int64_t>(64, n_events - e0);
        nb4[0] = as_const(off_a)[e0];
        nb4[1] = as_const(off_a)[e1];
        nb4[2] = as_const(off_b)[e0];
        nb4[3] = as_const(off_b)[e1];
    };
    int64_t t = static_cast<int64_t>(blockIdx.x) * MW + wave;
    if (t < n_tiles) bounds(t);
    for (; t < n_tiles; t += step) {
        const int64_t e0 = t * 64;
        const int ne = static_cast<int>(min<int64_t>(64, n_events - e0));
        const int64_t A0 = nb4[0], A1 = nb4[1], B0 = nb4[2], B1 = nb4[3];
        if (t + step < n_tiles) bounds(t + step);
        const int64_t e = e0 + lane;
        if (A1 - A0 > 64 * MKA || B1 - B0 > 64 * MKB) {
            // direct path: one lane per event, everything from HBM
            if (lane < ne) {
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
        // ---- every load of the tile in flight at once: buffer loads over
        // exactly the tile's ranges (0 past their ends, so no slot needs a
        // bounds test or a branch), raw bits converted after one wait
        const uint32_t ob = static_cast<uint32_t>(ne + 1) * 8u;
        const buf_t boa = buf_span(off_a + e0, ob), bob = buf_span(off_b + e0, ob);
        const uint32_t oa0 = buf_u32(boa, lane * 8), oa1 = buf_u32(boa, lane * 8 + 8);
        const uint32_t ob0 = buf_u32(bob, lane * 8), ob1 = buf_u32(bob, lane * 8 + 8);
        const uint32_t es = sizeof(T);
        const buf_t bea = buf_span(eta_a + A0, na * es), bpa = buf_span(phi_a + A0, na * es);
        const buf_t beb = buf_span(eta_b + B0, nb * es), bpb = buf_span(phi_b + B0, nb * es);
        uint32_t reb[MKB], rpb[MKB], rea[MKA], rpa[MKA];
#pragma unroll
        for (int k = 0; k < MKB; ++k) {
            reb[k] = buf_raw<T>(beb, lane + 64 * k);
            rpb[k] = buf_raw<T>(bpb, lane + 64 * k);
        }
#pragma unroll
        for (int k = 0; k < MKA; ++k) {
            rea[k] = buf_raw<T>(bea, lane + 64 * k);
            rpa[k] = buf_raw<T>(bpa, lane + 64 * k);
        }
        MaskWords<MBW> mwb{};
        MaskWords<MAW> mwa{};
        if (mask_b) mwb = mask_words<MBW>(mask_b + B0, nb, lane);
        if (mask_a) mwa = mask_words<MAW>(mask_a + A0, na, lane);
        asm volatile("" ::"v"(oa0), "v"(oa1), "v"(ob0), "v"(ob1));
#pragma unroll
        for (int k = 0; k < MKB; ++k) asm volatile("" ::"v"(reb[k]), "v"(rpb[k]));
#pragma unroll
        for (int k = 0; k < MKA; ++k) asm volatile("" ::"v"(rea[k]), "v"(rpa[k]));
#pragma unroll
        for (int k = 0; k < MBW; ++k) asm volatile("" ::"v"(mwb.v[k]));
#pragma unroll
        for (int k = 0; k < MAW; ++k) asm volatile("" ::"v"(mwa.v[k]));
        const bool in = lane < ne;
        const int32_t ab = in ? static_cast<int32_t>(oa0 - static_cast<uint32_t>(A0)) : 0;
        const int32_t ae = in ? static_cast<int32_t>(oa1 - static_cast<uint32_t>(A0)) : 0;
        const int32_t bb = in ? static_cast<int32_t>(ob0 - static_cast<uint32_t>(B0)) : 0;
        const int32_t bn = in ? static_cast<int32_t>(ob1 - static_cast<uint32_t>(B0)) - bb : 0;
        float veb[MKB], vpb[MKB], vea[MKA], vpa[MKA];
        bool oka[MKA];
#pragma unroll
        for (int k = 0; k < MKB; ++k) {
            veb[k] = raw_f<T>(reb[k]);
            vpb[k] = raw_f<T>(rpb[k]);
        }
#pragma unroll
        for (int k = 0; k < MKA; ++k) {
            vea[k] = raw_f<T>(rea[k]);
            vpa[k] = raw_f<T>(rpa[k]);
            oka[k] = true;
        }
        if (mask_b || mask_a) {
            const uint8_t *mbs = mask_b ? mask_stage<MBW>(mwb, mskb_s[wave], lane) : nullptr;
            const uint8_t *mas = mask_a ? mask_stage<MAW>(mwa, mska_s[wave], lane) : nullptr;
            wave_fence_dr();
            // a masked-out b gets eta = NaN: its dR^2 is NaN and never the minimum
#pragma unroll
            for (int k = 0; k < MKB; ++k)
                if (mask_b && lane + 64 * k < nb && !mbs[lane + 64 * k]) veb[k] = __builtin_nanf("");
#pragma unroll
            for (int k = 0; k < MKA; ++k)
                if (mask_a && lane + 64 * k < na) oka[k] = mas[lane + 64 * k] != 0;
        }
        // ---- b objects and the per-a b ranges into LDS
#pragma unroll
        for (int k = 0; k < MKB; ++k) {
            const int i = lane + 64 * k;
            if (i < nb) {
                be[i] = veb[k];
                bp[i] = vpb[k];
            }
        }
        if (lane < ne) {
            const uint32_t pk = static_cast<uint32_t>(bb) | (static_cast<uint32_t>(bn) << 16);
            int k = ab;
            for (; k + 2 <= ae; k += 2) {  // two per step: a divergent loop
                ar[k] = pk;
                ar[k + 1] = pk;
            }
            if (k < ae) ar[k] = pk;
        }
        wave_fence_dr();
        // ---- one lane per a object, slots in pairs: the pair's b ranges,
        // then the first two b objects of each range, each set of LDS reads
        // in flight together; only longer ranges loop over the rest.  A slot
        // past the tile's a objects reads a stale word (its range is not
        // used); reads past a range's end land in the next event's b objects
        // or the two padding entries and are not used either.
#pragma unroll
        for (int k0 = 0; k0 < MKA; k0 += 2) {
            uint32_t pk[2];
            float e0[2], p0[2], e1[2], p1[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) pk[u] = ar[lane + 64 * (k0 + u)];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int f = lane + 64 * (k0 + u) < na ? static_cast<int>(pk[u] & 0xffffu) : 0;
                e0[u] = be[f];
                p0[u] = bp[f];
                e1[u] = be[f + 1];
                p1[u] = bp[f + 1];
            }
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int k = k0 + u;
                const int i = lane + 64 * k;
                if (i < na) {
                    const int b0 = static_cast<int>(pk[u] & 0xffffu), nbk = static_cast<int>(pk[u] >> 16);
                    float best = INFINITY;
                    int32_t bi = -1;
                    // ascending order with a strict '<': the lowest index wins ties
                    if (nbk >= 1) {
                        const float d2 = delta_r2(vea[k], vpa[k], e0[u], p0[u]);
                        if (d2 < best) {
                            best = d2;
                            bi = 0;
                        }
                    }
                    if (nbk >= 2) {
                        const float d2 = delta_r2(vea[k], vpa[k], e1[u], p1[u]);
                        if (d2 < best) {
                            best = d2;
                            bi = 1;
                        }
                    }
                    for (int b = b0 + 2; b < b0 + nbk; ++b) {
                        const float d2 = delta_r2(vea[k], vpa[k], be[b], bp[b]);
                        if (d2 < best) {
                            best = d2;
                            bi = b - b0;
                        }
                    }
                    const int64_t a = A0 + i;
                    if (min_dr2) min_dr2[a] = best;
                    if (idx_b) idx_b[a] = bi;
                    if (clean) clean[a] = (oka[k] && !(best <= thr2)) ? 1 : 0;
                }
            }
        }
        wave_fence_dr();  // the next tile overwrites the staging
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
    const int64_t n_tiles = ceil_div(n_events, 64);
    const int grid = static_cast<int>(std::min<int64_t>(ceil_div(n_tiles, MW), kTileWgPerCu * device_cus()));
    if (dtype == HEPK_F16)
        match_dr_kernel<_Float16><<<grid, 64 * MW, 0, stream>>>(
            off_a, static_cast<const _Float16 *>(eta_a), static_cast<const _Float16 *>(phi_a), mask_a, off_b,
            static_cast<const _Float16 *>(eta_b), static_cast<const _Float16 *>(phi_b), mask_b, n_events, thr2,
            min_dr2, idx_b, clean_out);
    else
        match_dr_kernel<float><<<grid, 64 * MW, 0, stream>>>(
            off_a, static_cast<const float *>(eta_a), static_cast<const float *>(phi_a), mask_a, off_b,
            static_cast<const float *>(eta_b), static_cast<const float *>(phi_b), mask_b, n_events, thr2,
            min_dr2, idx_b, clean_out);
    return check_launch("hepk_match_dr");
}
