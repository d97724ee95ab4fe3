// Top-quark candidate reconstruction (Sec. IV high-level variable
// reconstruction: the jet triplet whose invariant mass is closest to
// M = 172 GeV).
//
// hepk_p4 turns (pt, eta, phi, mass) into Cartesian four-momenta
// (elementwise).  hepk_best_triplet searches, per event, every triplet of
// selected objects.  The work per event grows as C(n, 3), so one lane per
// event would leave most lanes of a wavefront idle behind its densest event;
// instead each wavefront owns tiles of 64 consecutive events and spreads the
// tile's triplets evenly over its 64 lanes:
//   1. the tile's objects are loaded with all loads in flight, and the
//      selected ones compacted by wavefront ballot into LDS (four-momenta and
//      index in the tile), so each event's selected objects are contiguous;
//   2. the events' triplet counts C(n_e, 3) are prefix-summed across the
//      wavefront;
//   3. lane l takes the l-th 1/64 of the tile's triplets in lexicographic
//      order (i < j < k within an event, events in order), finds its first
//      triplet by a search over the prefix sums and the combinatorial number
//      system, and walks on from there;
//   4. per triplet: three float32 sums per component (the pair sum of i and
//      j kept while only k moves), the mass square
//      E^2 - px^2 - py^2 - pz^2 (each product and difference rounded on its
//      own), a correctly rounded square root and the distance d to the
//      target; a lane keeps the smallest (d, rank in the event) and merges it
//      with an LDS 64-bit atomic minimum when it leaves an event, which keeps
//      the first triplet in order on ties (a NaN or infinite d is never
//      taken);
//   5. each event lane turns its minimum back into (i, j, k) and recomputes
//      the mass with the same operations.
// Tiles with more objects than the LDS staging holds search their events one
// lane per event straight from HBM.
#include "common.hpp"

namespace hepk {

constexpr int TB = 256;
constexpr int TWV = TB / 64;
// objects per lane staged for a tile (384 per tile: 3.6 standard deviations
// above the 320 jets of 64 events of the analysis workloads; 9.1 KB of LDS
// per wavefront, so four wavefronts per SIMD instead of three with 512)
constexpr int TK = 6;

__device__ __forceinline__ void p4_one(float p, float h, float f, float m, float &x, float &y, float &z, float &e) {
    float s, c;
    sincosf(f, &s, &c);
    x = p * c, y = p * s, z = p * sinhf(h);
    const float xx = x * x, yy = y * y, zz = z * z, mm = m * m;
    e = sqrtf(((xx + yy) + zz) + mm);
}

__global__ __launch_bounds__(256) void p4_kernel(const float *__restrict__ pt, const float *__restrict__ eta,
                                                 const float *__restrict__ phi, const float *__restrict__ mass,
                                                 int64_t n, float *__restrict__ px, float *__restrict__ py,
                                                 float *__restrict__ pz, float *__restrict__ en) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride)
        p4_one(pt[i], eta[i], phi[i], mass[i], px[i], py[i], pz[i], en[i]);
}

// Up to 64 workgroups per CU (a sweep of 8-64: 64 best; with nontemporal
// loads and stores, every byte touched once: 312 -> 284 us on 5e7 jets).
constexpr int kP4WgPerCu = 64;
typedef float p4f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ p4f32x4 p4ld(const float *p, int64_t q) {
    return __builtin_nontemporal_load(reinterpret_cast<const p4f32x4 *>(p) + q);
}
__device__ __forceinline__ void p4st(p4f32x4 v, float *p, int64_t q) {
    __builtin_nontemporal_store(v, reinterpret_cast<p4f32x4 *>(p) + q);
}

// Four consecutive objects per thread and step (all eight columns 16-byte
// aligned): one 16-byte load per input column and one 16-byte store per
// output column; the n % 4 last objects one per thread.
__global__ __launch_bounds__(256) void p4_vec4_kernel(const float *__restrict__ pt, const float *__restrict__ eta,
                                                      const float *__restrict__ phi, const float *__restrict__ mass,
                                                      int64_t n, float *__restrict__ px, float *__restrict__ py,
                                                      float *__restrict__ pz, float *__restrict__ en) {
    const int64_t n4 = n / 4;
    const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
    const int64_t gid = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (gid < n - 4 * n4) {
        const int64_t i = 4 * n4 + gid;
        p4_one(pt[i], eta[i], phi[i], mass[i], px[i], py[i], pz[i], en[i]);
    }
    for (int64_t q = gid; q < n4; q += stride) {
        const p4f32x4 p = p4ld(pt, q), h = p4ld(eta, q), f = p4ld(phi, q), m = p4ld(mass, q);
        float xs[4], ys[4], zs[4], es[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) p4_one(p[j], h[j], f[j], m[j], xs[j], ys[j], zs[j], es[j]);
        const p4f32x4 x = {xs[0], xs[1], xs[2], xs[3]}, y = {ys[0], ys[1], ys[2], ys[3]};
        const p4f32x4 z = {zs[0], zs[1], zs[2], zs[3]}, e = {es[0], es[1], es[2], es[3]};
        p4st(x, px, q);
        p4st(y, py, q);
        p4st(z, pz, q);
        p4st(e, en, q);
    }
}

__device__ __forceinline__ void wave_fence_t() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Running best triplet of one event.
struct Best {
    float d = INFINITY, m = __builtin_nanf("");
    int32_t i = -1, j = -1, k = -1;
};

// Triplets of the selected objects among [0, n) of the arrays X/Y/Z/E (LDS
// or HBM), local indices relative to `first`.
template <typename P, typename M>
__device__ __forceinline__ Best search(const P &X, const P &Y, const P &Z, const P &E, const M &sel, int64_t first,
                                       int64_t n, float target) {
    Best b;
    for (int64_t i = 0; i < n; ++i) {
        if (!sel(first + i)) continue;
        const float xi = X[first + i], yi = Y[first + i], zi = Z[first + i], ei = E[first + i];
        for (int64_t j = i + 1; j < n; ++j) {
            if (!sel(first + j)) continue;
            const float xij = xi + X[first + j], yij = yi + Y[first + j];
            const float zij = zi + Z[first + j], eij = ei + E[first + j];
            for (int64_t k = j + 1; k < n; ++k) {
                if (!sel(first + k)) continue;
                const float sx = xij + X[first + k], sy = yij + Y[first + k];
                const float sz = zij + Z[first + k], se = eij + E[first + k];
                float m2 = se * se;
                m2 = m2 - sx * sx;
                m2 = m2 - sy * sy;
                m2 = m2 - sz * sz;
                // a negative square (rounding of a light system) is mass 0; NaN stays NaN
                const float mm = (m2 < 0.0f) ? 0.0f : sqrtf(m2);
                const float d = fabsf(mm - target);
                if (d < b.d) {
                    b.d = d;
                    b.m = mm;
                    b.i = static_cast<int32_t>(i);
                    b.j = static_cast<int32_t>(j);
                    b.k = static_cast<int32_t>(k);
                }
            }
        }
    }
    return b;
}

// Triplets with first index i among n objects: C(n - i - 1, 2).
__device__ __forceinline__ int64_t c2(int64_t m) { return m * (m - 1) / 2; }
__device__ __forceinline__ int64_t c3(int64_t m) { return m * (m - 1) * (m - 2) / 6; }

// Mass of a triplet and its distance to the target (the arithmetic of the
// search; NaN stays NaN).
__device__ __forceinline__ void triplet_mass(const float *X, const float *Y, const float *Z, const float *E, int i, int j,
                                             int k, float target, float &mm, float &d) {
    const float sx = (X[i] + X[j]) + X[k], sy = (Y[i] + Y[j]) + Y[k];
    const float sz = (Z[i] + Z[j]) + Z[k], se = (E[i] + E[j]) + E[k];
    float m2 = se * se;
    m2 = m2 - sx * sx;
    m2 = m2 - sy * sy;
    m2 = m2 - sz * sz;
    mm = (m2 < 0.0f) ? 0.0f : sqrtf(m2);
    d = fabsf(mm - target);
}

// (i, j, k) of the triplet of lexicographic rank r among n objects.
__device__ __forceinline__ void unrank(int64_t r, int n, int &i, int &j, int &k) {
    i = 0;
    while (r >= c2(n - i - 1)) {
        r -= c2(n - i - 1);
        ++i;
    }
    j = i + 1;
    while (r >= n - j - 1) {
        r -= n - j - 1;
        ++j;
    }
    k = j + 1 + static_cast<int>(r);
}

struct TripletLds {
    float x[64 * TK], y[64 * TK], z[64 * TK], e[64 * TK];  // selected objects, compacted
    uint16_t li[64 * TK];                                  // their index in the tile
    uint16_t pre[64 * TK + 1];                             // selected objects before each object
    int64_t tp[65];                                        // triplets of the events before each
    uint64_t key[64];                                      // per event: min (d bits << 32 | rank)
    int32_t s0[64], n[64];                                 // per event: first selected, count
};

__global__ __launch_bounds__(TB) void best_triplet_kernel(const int64_t *__restrict__ off, int64_t n_events,
                                                          const float *__restrict__ px, const float *__restrict__ py,
                                                          const float *__restrict__ pz, const float *__restrict__ en,
                                                          const uint8_t *__restrict__ om, float target,
                                                          float *__restrict__ out_mass, int32_t *__restrict__ out_idx) {
    __shared__ TripletLds lds[TWV];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    TripletLds &L = lds[wave];
    const int64_t n_tiles = ceil_div(n_events, 64);
    const int64_t step = static_cast<int64_t>(gridDim.x) * TWV;
    for (int64_t t = static_cast<int64_t>(blockIdx.x) * TWV + wave; t < n_tiles; t += step) {
        const int64_t e0 = t * 64;
        const int ne = static_cast<int>(min<int64_t>(64, n_events - e0));
        const int64_t A = as_const(off)[e0];
        const int64_t tot = as_const(off)[e0 + ne] - A;
        const int64_t e = e0 + lane;
        const bool act = lane < ne;
        int64_t a0 = 0, a1 = 0;
        if (act) {
            a0 = off[e] - A;
            a1 = off[e + 1] - A;
        }
        if (tot > 64 * TK) {
            // dense tile: one lane per event from HBM
            Best b;
            if (act) {
                auto sel = [&](int64_t i) { return !om || om[A + i] != 0; };
                b = search(px + A, py + A, pz + A, en + A, sel, a0, a1 - a0, target);
                out_mass[e] = b.m;
                out_idx[3 * e] = b.i;
                out_idx[3 * e + 1] = b.j;
                out_idx[3 * e + 2] = b.k;
            }
            continue;
        }
        // 1. loads (buffer loads over exactly the tile's objects: 0 past the
        // end, no per-slot branch, all in flight and waited for once), then
        // the selected objects compacted in tile order
        const int nobj = static_cast<int>(tot);
        const uint32_t nb4 = static_cast<uint32_t>(nobj) * 4u;
        const buf_t bx = buf_span(px + A, nb4), by = buf_span(py + A, nb4);
        const buf_t bz = buf_span(pz + A, nb4), be = buf_span(en + A, nb4);
        const buf_t bm = buf_span(om ? static_cast<const void *>(om + A) : static_cast<const void *>(px),
                                  om ? static_cast<uint32_t>(nobj) : 0u);
        float vx[TK], vy[TK], vz[TK], ve[TK];
        uint32_t mk[TK];
        bool sel[TK];
#pragma unroll
        for (int k = 0; k < TK; ++k) {
            const int i = lane + 64 * k;
            vx[k] = __builtin_bit_cast(float, buf_u32<kBufNt>(bx, i * 4));
            vy[k] = __builtin_bit_cast(float, buf_u32<kBufNt>(by, i * 4));
            vz[k] = __builtin_bit_cast(float, buf_u32<kBufNt>(bz, i * 4));
            ve[k] = __builtin_bit_cast(float, buf_u32<kBufNt>(be, i * 4));
            mk[k] = om ? __builtin_amdgcn_raw_buffer_load_b8(bm, i, 0, kBufNt) : 1u;
        }
#pragma unroll
        for (int k = 0; k < TK; ++k) asm volatile("" ::"v"(vx[k]), "v"(vy[k]), "v"(vz[k]), "v"(ve[k]), "v"(mk[k]));
#pragma unroll
        for (int k = 0; k < TK; ++k) sel[k] = (lane + 64 * k < nobj) & (mk[k] != 0u);
        int run = 0;
#pragma unroll
        for (int k = 0; k < TK; ++k) {
            const int i = lane + 64 * k;
            const uint64_t bal = __ballot(sel[k]);
            const int before = run + static_cast<int>(__builtin_amdgcn_mbcnt_hi(
                                         static_cast<uint32_t>(bal >> 32),
                                         __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(bal), 0u)));
            if (i < nobj) L.pre[i] = static_cast<uint16_t>(before);
            if (sel[k]) {
                L.x[before] = vx[k];
                L.y[before] = vy[k];
                L.z[before] = vz[k];
                L.e[before] = ve[k];
                L.li[before] = static_cast<uint16_t>(i);
            }
            run += __popcll(bal);
        }
        if (lane == 0) L.pre[nobj] = static_cast<uint16_t>(run);
        wave_fence_t();
        // 2. per event: first selected object, count, triplets; prefix sums
        // over the tile
        int s0 = 0, nn = 0;
        if (act) {
            s0 = L.pre[a0];
            nn = L.pre[a1] - s0;
        }
        const int64_t tcount = act ? c3(nn) : 0;
        int64_t incl = tcount;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t up = __shfl_up(incl, d, 64);
            if (lane >= d) incl += up;
        }
        L.tp[lane + 1] = incl;
        if (lane == 0) L.tp[0] = 0;
        L.s0[lane] = s0;
        L.n[lane] = nn;
        L.key[lane] = ~0ull;
        wave_fence_t();
        // 3-4. this lane's share of the tile's triplets
        const int64_t T = L.tp[64];
        const int64_t t0 = T * lane / 64, t1 = T * (lane + 1) / 64;
        if (t0 < t1) {
            int ev = 0;  // the last event with tp[ev] <= t0
            for (int lo = 0, hi = 63; lo <= hi;) {
                const int mid = (lo + hi) >> 1;
                if (L.tp[mid] <= t0) {
                    ev = mid;
                    lo = mid + 1;
                } else {
                    hi = mid - 1;
                }
            }
            while (L.tp[ev + 1] <= t0) ++ev;  // skip events without triplets
            int n = L.n[ev], base = L.s0[ev];
            int64_t rank = t0 - L.tp[ev];
            int i, j, k;
            unrank(rank, n, i, j, k);
            uint64_t best = ~0ull;
            // the pair sums (X[i] + X[j]) of the current (i, j), reread only
            // when i or j moves: the same value the mass adds X[k] to
            float pxij = L.x[base + i] + L.x[base + j], pyij = L.y[base + i] + L.y[base + j];
            float pzij = L.z[base + i] + L.z[base + j], peij = L.e[base + i] + L.e[base + j];
            for (int64_t tt = t0; tt < t1; ++tt) {
                const float sx = pxij + L.x[base + k], sy = pyij + L.y[base + k];
                const float sz = pzij + L.z[base + k], se = peij + L.e[base + k];
                float m2 = se * se;
                m2 = m2 - sx * sx;
                m2 = m2 - sy * sy;
                m2 = m2 - sz * sz;
                const float mm = (m2 < 0.0f) ? 0.0f : sqrtf(m2);
                const float d = fabsf(mm - target);
                if (d < INFINITY) {  // NaN and infinite distances are never taken
                    const uint64_t key = (static_cast<uint64_t>(__float_as_uint(d)) << 32) | static_cast<uint64_t>(rank);
                    best = key < best ? key : best;
                }
                // next triplet in order
                ++rank;
                if (++k == n) {
                    if (++j == n - 1) {
                        if (++i == n - 2) {
                            // the event is done: merge and move to the next with triplets
                            if (best != ~0ull) atomicMin(reinterpret_cast<unsigned long long *>(&L.key[ev]), best);
                            best = ~0ull;
                            if (tt + 1 < t1) {
                                do {
                                    ++ev;
                                } while (L.tp[ev + 1] == L.tp[ev]);
                                n = L.n[ev];
                                base = L.s0[ev];
                            }
                            i = 0;
                            rank = 0;
                        }
                        j = i + 1;
                    }
                    k = j + 1;
                    pxij = L.x[base + i] + L.x[base + j];
                    pyij = L.y[base + i] + L.y[base + j];
                    pzij = L.z[base + i] + L.z[base + j];
                    peij = L.e[base + i] + L.e[base + j];
                }
            }
            if (best != ~0ull) atomicMin(reinterpret_cast<unsigned long long *>(&L.key[ev]), best);
        }
        wave_fence_t();
        // 5. each event's minimum back to its triplet and mass
        if (act) {
            const uint64_t key = L.key[lane];
            float mm = __builtin_nanf("");
            int32_t bi = -1, bj = -1, bk = -1;
            if (key != ~0ull) {
                int i, j, k;
                unrank(static_cast<int64_t>(key & 0xffffffffu), nn, i, j, k);
                float d;
                triplet_mass(L.x + s0, L.y + s0, L.z + s0, L.e + s0, i, j, k, target, mm, d);
                // local index = tile index of the compacted object - the event's first
                bi = static_cast<int32_t>(L.li[s0 + i]) - static_cast<int32_t>(a0);
                bj = static_cast<int32_t>(L.li[s0 + j]) - static_cast<int32_t>(a0);
                bk = static_cast<int32_t>(L.li[s0 + k]) - static_cast<int32_t>(a0);
            }
            out_mass[e] = mm;
            out_idx[3 * e] = bi;
            out_idx[3 * e + 1] = bj;
            out_idx[3 * e + 2] = bk;
        }
        wave_fence_t();  // the next tile overwrites the staging
    }
}

}  // namespace hepk

extern "C" int hepk_p4(const float *pt, const float *eta, const float *phi, const float *mass, int64_t n, float *px,
                       float *py, float *pz, float *en, hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(n >= 0, "hepk_p4: n < 0");
    HEPK_REQUIRE(n == 0 || (pt && eta && phi && mass && px && py && pz && en), "hepk_p4: NULL column");
    if (n == 0) return HEPK_OK;
    bool al = true;
    for (const void *p : {static_cast<const void *>(pt), static_cast<const void *>(eta), static_cast<const void *>(phi),
                          static_cast<const void *>(mass), static_cast<const void *>(px), static_cast<const void *>(py),
                          static_cast<const void *>(pz), static_cast<const void *>(en)})
        al = al && reinterpret_cast<uintptr_t>(p) % 16 == 0;
    if (al) {
        const int g = static_cast<int>(
            std::max<int64_t>(1, std::min<int64_t>(ceil_div(n / 4, 256), kP4WgPerCu * device_cus())));
        p4_vec4_kernel<<<g, 256, 0, stream>>>(pt, eta, phi, mass, n, px, py, pz, en);
        return check_launch("hepk_p4");
    }
    const int g = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 16 * device_cus())));
    p4_kernel<<<g, 256, 0, stream>>>(pt, eta, phi, mass, n, px, py, pz, en);
    return check_launch("hepk_p4");
}

extern "C" int hepk_best_triplet(const int64_t *offsets, int64_t n_events, const float *px, const float *py,
                                 const float *pz, const float *en, const uint8_t *obj_mask, float target,
                                 float *out_mass, int32_t *out_idx, hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(n_events >= 0 && offsets, "hepk_best_triplet: bad offsets or n_events");
    HEPK_REQUIRE(n_events == 0 || (px && py && pz && en && out_mass && out_idx), "hepk_best_triplet: NULL array");
    if (n_events == 0) return HEPK_OK;
    const int g = static_cast<int>(
        std::max<int64_t>(1, std::min<int64_t>(ceil_div(ceil_div(n_events, 64), TWV), 16 * device_cus())));
    best_triplet_kernel<<<g, TB, 0, stream>>>(offsets, n_events, px, py, pz, en, obj_mask, target, out_mass,
                                              out_idx);
    return check_launch("hepk_best_triplet");
}
