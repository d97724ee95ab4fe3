// Top-quark candidate reconstruction (Sec. IV high-level variable
// reconstruction: the jet triplet whose invariant mass is closest to
// M = 172 GeV).
//
// hepk_p4 turns (pt, eta, phi, mass) into Cartesian four-momenta
// (elementwise).  hepk_best_triplet searches, per event, every triplet of
// selected objects: each wavefront owns tiles of 64 consecutive events,
// stages the tile's four-momenta and mask in its LDS with all loads in
// flight, and one lane per event runs over its triplets (i < j < k) in
// order, the pair sum i + j held while k runs.  Per triplet: three float32
// sums per component, the mass square E^2 - px^2 - py^2 - pz^2 (each product
// and difference rounded on its own), a correctly rounded square root and
// the distance to the target; a strict '<' keeps the first triplet on ties.
// The search is the first part of the analysis whose work grows faster than
// its input (C(n, 3) triplets for n jets).  Tiles with more objects than the
// LDS staging holds walk their events straight from HBM.
#include "common.hpp"

namespace hepk {

constexpr int TB = 256;
constexpr int TWV = TB / 64;
constexpr int TK = 8;  // objects per lane staged for a tile (512 per tile)

__global__ __launch_bounds__(256) void p4_kernel(const float *__restrict__ pt, const float *__restrict__ eta,
                                                 const float *__restrict__ phi, const float *__restrict__ mass,
                                                 int64_t n, float *__restrict__ px, float *__restrict__ py,
                                                 float *__restrict__ pz, float *__restrict__ en) {
    const int64_t stride = static_cast<int64_t>(gridDim.x) * 256;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; i < n; i += stride) {
        const float p = pt[i], h = eta[i], f = phi[i], m = mass[i];
        float s, c;
        sincosf(f, &s, &c);
        const float x = p * c, y = p * s, z = p * sinhf(h);
        const float xx = x * x, yy = y * y, zz = z * z, mm = m * m;
        px[i] = x;
        py[i] = y;
        pz[i] = z;
        en[i] = sqrtf(((xx + yy) + zz) + mm);
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

__global__ __launch_bounds__(TB) void best_triplet_kernel(const int64_t *__restrict__ off, int64_t n_events,
                                                          const float *__restrict__ px, const float *__restrict__ py,
                                                          const float *__restrict__ pz, const float *__restrict__ en,
                                                          const uint8_t *__restrict__ om, float target,
                                                          float *__restrict__ out_mass, int32_t *__restrict__ out_idx) {
    __shared__ float sx[TWV][64 * TK], sy[TWV][64 * TK], sz[TWV][64 * TK], se[TWV][64 * TK];
    __shared__ uint8_t sm[TWV][64 * TK];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
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
        Best b;
        if (tot <= 64 * TK) {
            const int n = static_cast<int>(tot);
            float vx[TK], vy[TK], vz[TK], ve[TK];
            uint8_t vm[TK];
#pragma unroll
            for (int k = 0; k < TK; ++k) {
                const int i = lane + 64 * k;
                vx[k] = vy[k] = vz[k] = ve[k] = 0.0f;
                vm[k] = 0;
                if (i < n) {
                    vx[k] = px[A + i];
                    vy[k] = py[A + i];
                    vz[k] = pz[A + i];
                    ve[k] = en[A + i];
                    vm[k] = om ? om[A + i] : 1;
                }
            }
#pragma unroll
            for (int k = 0; k < TK; ++k) {
                const int i = lane + 64 * k;
                if (i < n) {
                    sx[wave][i] = vx[k];
                    sy[wave][i] = vy[k];
                    sz[wave][i] = vz[k];
                    se[wave][i] = ve[k];
                    sm[wave][i] = vm[k];
                }
            }
            wave_fence_t();
            if (act) {
                const uint8_t *msk = sm[wave];
                auto sel = [&](int64_t i) { return msk[i] != 0; };
                b = search(sx[wave], sy[wave], sz[wave], se[wave], sel, a0, a1 - a0, target);
            }
            wave_fence_t();  // the next tile overwrites the staging
        } else if (act) {
            auto sel = [&](int64_t i) { return !om || om[A + i] != 0; };
            const float *X = px + A, *Y = py + A, *Z = pz + A, *E = en + A;
            b = search(X, Y, Z, E, sel, a0, a1 - a0, target);
        }
        if (act) {
            out_mass[e] = b.m;
            out_idx[3 * e] = b.i;
            out_idx[3 * e + 1] = b.j;
            out_idx[3 * e + 2] = b.k;
        }
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
