// hepk_pipeline: the whole analysis pass of Sec. IV (object selection,
// lepton-jet Delta-R cleaning, per-event reductions, event selection,
// weighted histograms, jet-energy-scale variations) fused into one
// persistent kernel, for any number of datasets and queries at once.
//
// Sec. IV observes that hundreds of small kernel calls per pass left the GPU
// half idle and names fusion as the fix; here every intermediate (object
// masks, per-event counts and sums, event masks) lives in registers and LDS,
// so a pass reads each input column from HBM once and writes only the
// histograms.
//
// Work decomposition.  Each wavefront owns tiles of TW = 64 * EVPL
// consecutive events and works through them without waiting for the other
// wavefronts of its workgroup (no workgroup barrier inside a tile: the four
// or eight wavefronts of a workgroup only share the LDS histograms, updated
// with atomics).  The host cuts every dataset's tiles into chunks; a
// workgroup takes whole chunks, so a chunk never mixes datasets and the LDS
// histograms are merged into HBM only when the workgroup moves to another
// dataset.  For one tile a wavefront
//   1. reads the tile's object ranges with scalar loads, then issues all of
//      its loads at once -- offsets and weight of its events, up to JK jets,
//      MK muons and EK electrons per lane (consecutive lanes, consecutive
//      objects: coalesced) -- into registers, and waits once;
//   2. puts the offsets in LDS (tile-relative int32) and lets each event lane
//      write its event index over its jets (the jet -> event map);
//   3. per query: muon lanes evaluate the muon cuts and stage eta/phi in LDS,
//      eta = NaN for muons that fail (a NaN dR^2 never passes the cone test,
//      which is the same as skipping them); electrons likewise;
//   4. jet lanes test the cone against their event's staged leptons and store
//      pt (or NaN when removed or outside |eta|) in LDS;
//   5. event lanes walk their jets in order for each jet-energy scale s:
//      ptv = pt * s, the jet cut, the count, the left-to-right float32 H_T,
//      the maximum, the b-tag count; then the event cut and three fills into
//      the workgroup's LDS histograms (float64 sums, uint32 counts).
// Steps 2-5 exchange data through the wavefront's own LDS region; a
// wavefront's LDS operations complete in issue order, so only compiler
// ordering fences are needed between them.  A tile whose objects exceed the
// register capacity (a 5-sigma fluctuation for the paper's multiplicities,
// always possible for arbitrary input) is processed one lane per event
// straight from HBM with the same arithmetic.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"

namespace hepk {

struct DsDev {
    int64_t n_events;
    const int64_t *joff, *moff, *eoff;
    const void *jpt, *jeta, *jphi, *jbt;
    const void *mpt, *meta, *mphi, *miso;
    const void *ept, *eeta, *ephi;
    const float *w;
    int64_t hist0;  // first slot of this dataset's block of histograms
};

struct QDev {
    float mu_pt, mu_abseta, mu_iso, el_pt, el_abseta, jet_pt, jet_abseta, thr2, btag;
    int32_t min_mu, min_jet, min_b;
    int32_t n_scale, scale0;
    int32_t active;      // 0: idle query slot, skipped
    int32_t nbins[3];
    int32_t ebase[3];    // first edge of each observable in the plan's edge table
    float lo[3], hi[3];  // first and last edge of each observable
    float inv_w[3];      // nbins / (hi - lo): start value of the bin search
    // Histogram of (scale v, observable h) starts at slot0 + v * per_scale +
    // hoff[h]: in the workgroup's LDS copy (compact over the active queries)
    // and in the dataset's block in HBM (fixed per query slot).
    int32_t lslot0, lper_scale, lhoff[3];
    int32_t gslot0, gper_scale, ghoff[3];
};

struct Chunk {
    int32_t d, pad;
    int64_t t0, t1;  // tiles [t0, t1) of dataset d
};

struct PipeArgs {
    const DsDev *ds;
    const QDev *qs;
    const float *scales;
    const Chunk *chunks;
    const float *edges;  // all queries' bin edges, concatenated
    int32_t chunk_begin, chunk_end;  // chunks [chunk_begin, chunk_end) of `chunks`
    int32_t n_q, ds_slots, n_edges, edges_in_lds;  // ds_slots: LDS histogram slots
    double *sumw;
    uint64_t *counts;
};

template <bool LDSH>
struct HistSink {
    double *sw;        // LDS (LDSH) or the dataset's block in HBM
    uint32_t *c32;     // LDS (LDSH)
    uint64_t *c64;     // HBM (!LDSH)

    __device__ __forceinline__ void add(int slot, double w) const {
        if (LDSH) {
            atomic_add_f64(&sw[slot], w);
            atomicAdd(&c32[slot], 1u);
        } else {
            atomic_add_f64(&sw[slot], w);
            atomic_add_u64(&c64[slot], 1u);
        }
    }
};

// Fills H_T, lead and nJet of one passing event for scale v of query Q (a
// table entry read in place, so its fields are fetched where they are used).
template <bool LDSH, typename QT>
__device__ __forceinline__ void fill3(const HistSink<LDSH> &sink, const QT &Q, const float *edges, int v,
                                      float ht, float lead, int nj, double w) {
    const int base = LDSH ? Q.lslot0 + v * Q.lper_scale : Q.gslot0 + v * Q.gper_scale;
    const float xs[3] = {ht, lead, static_cast<float>(nj)};
#pragma unroll
    for (int h = 0; h < 3; ++h) {
        const float x = xs[h];
        if (x != x) continue;
        const int s = hist_slot_lohi(x, edges + Q.ebase[h], Q.nbins[h], Q.lo[h], Q.hi[h], Q.inv_w[h]);
        sink.add(base + (LDSH ? Q.lhoff[h] : Q.ghoff[h]) + s, w);
    }
}

// Orders this wavefront's LDS accesses around the point (LDS executes one
// wavefront's operations in issue order, so no wait is needed, only that the
// compiler keeps the order).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One event, one lane, columns read straight from HBM.
template <typename T, bool EXT, bool LDSH>
__device__ void event_direct(const PipeArgs &P, const DsDev &D, int64_t e, const float *edges,
                             const HistSink<LDSH> &sink) {
    const bool has_iso = D.miso != nullptr;
    const bool has_el = EXT && D.eoff != nullptr;
    const bool has_bt = EXT && D.jbt != nullptr;
    const double w = D.w ? static_cast<double>(D.w[e]) : 1.0;
    const int64_t j0 = D.joff[e], j1 = D.joff[e + 1];
    const int64_t m0 = D.moff[e], m1 = D.moff[e + 1];
    const int64_t l0 = has_el ? D.eoff[e] : 0, l1 = has_el ? D.eoff[e + 1] : 0;
    const T *jpt = static_cast<const T *>(D.jpt), *jeta = static_cast<const T *>(D.jeta);
    const T *jphi = static_cast<const T *>(D.jphi), *jbt = static_cast<const T *>(D.jbt);
    const T *mpt = static_cast<const T *>(D.mpt), *meta = static_cast<const T *>(D.meta);
    const T *mphi = static_cast<const T *>(D.mphi), *miso = static_cast<const T *>(D.miso);
    const T *ept = static_cast<const T *>(D.ept), *eeta = static_cast<const T *>(D.eeta);
    const T *ephi = static_cast<const T *>(D.ephi);
    for (int q = 0; q < P.n_q; ++q) {
        const QDev Q = as_const(P.qs)[q];
        if (!Q.active) continue;
        auto mu_sel = [&](int64_t m) {
            return ldf(mpt, m) > Q.mu_pt && fabsf(ldf(meta, m)) < Q.mu_abseta &&
                   (!has_iso || ldf(miso, m) < Q.mu_iso);
        };
        auto el_sel = [&](int64_t m) { return ldf(ept, m) > Q.el_pt && fabsf(ldf(eeta, m)) < Q.el_abseta; };
        int nmu = 0;
        for (int64_t m = m0; m < m1; ++m) nmu += mu_sel(m) ? 1 : 0;
        for (int v = 0; v < Q.n_scale; ++v) {
            const float s = as_const(P.scales)[Q.scale0 + v];
            int nj = 0, nb = 0;
            float ht = 0.0f, lead = -INFINITY;
            for (int64_t j = j0; j < j1; ++j) {
                const float x = ldf(jpt, j) * s;
                const float eta = ldf(jeta, j);
                if (!(x > Q.jet_pt && fabsf(eta) < Q.jet_abseta)) continue;
                const float phi = ldf(jphi, j);
                bool hit = false;
                for (int64_t m = m0; m < m1 && !hit; ++m)
                    hit = mu_sel(m) && delta_r2(eta, phi, ldf(meta, m), ldf(mphi, m)) <= Q.thr2;
                for (int64_t m = l0; m < l1 && !hit; ++m)
                    hit = el_sel(m) && delta_r2(eta, phi, ldf(eeta, m), ldf(ephi, m)) <= Q.thr2;
                if (hit) continue;
                if (nj == 0 || x > lead) lead = x;
                ++nj;
                ht = ht + x;
                if (has_bt && ldf(jbt, j) > Q.btag) ++nb;
            }
            const bool pass = nmu >= Q.min_mu && nj >= Q.min_jet && (!has_bt || nb >= Q.min_b);
            if (pass) fill3(sink, Q, edges, v, ht, lead, nj, w);
        }
    }
}

template <int EVPL, bool EXT>
struct Caps {
    static constexpr int TW = 64 * EVPL;             // events per wavefront tile
    static constexpr int JK = 6 * EVPL + 1;          // jet slots per lane
    static constexpr int MK = 2 * EVPL + 1;          // muon slots per lane
    static constexpr int EK = EXT ? 2 * EVPL : 1;    // electron slots per lane
    static constexpr int JC = 64 * JK, MC = 64 * MK, EC = 64 * EK;
};

// One wavefront's LDS.  jr holds, per jet, its event's range of selected
// muons (first | count << 16) until the cone test reads it; the same word
// then holds the jet's pt (or NaN) for the per-event walk.
template <int EVPL, bool EXT>
struct WaveLds {
    using C = Caps<EVPL, EXT>;
    union {
        uint32_t rng;
        float pt;
    } jr[C::JC];
    uint32_t jre[EXT ? C::JC : 1];   // same for selected electrons
    float seta[C::MC], sphi[C::MC];  // selected muons, compacted in tile order
    float sea[EXT ? C::EC : 1], sep[EXT ? C::EC : 1];
    uint16_t mpre[C::MC + 1];        // selected muons before muon m
    uint16_t epre[EXT ? C::EC + 1 : 1];
    uint8_t bt[EXT ? C::JC : 1];
    // per event, for queries with several jet-energy scales: jet range
    // (first | end << 16), selected muons, weight
    uint32_t evjr[C::TW];
    uint16_t evnmu[C::TW];
    float evw[C::TW];
};

struct TileBounds {
    int64_t J0, J1, M0, M1, L0, L1;
};

template <bool EXT, typename DT>
__device__ __forceinline__ TileBounds tile_bounds(const DT &D, bool has_el, int64_t e0, int ne) {
    TileBounds b;
    b.J0 = as_const(D.joff)[e0];
    b.J1 = as_const(D.joff)[e0 + ne];
    b.M0 = as_const(D.moff)[e0];
    b.M1 = as_const(D.moff)[e0 + ne];
    b.L0 = (EXT && has_el) ? as_const(D.eoff)[e0] : 0;
    b.L1 = (EXT && has_el) ? as_const(D.eoff)[e0 + ne] : 0;
    return b;
}

// Compacts the selected objects of a tile (sel per slot k of this lane) into
// (eta, phi) arrays in tile order; pre[m] = number of selected objects before
// object m, pre[n] = total.
template <int K>
__device__ __forceinline__ void compact(const bool (&sel)[K], const float (&eta)[K], const float (&phi)[K], int n,
                                        int lane, float *oeta, float *ophi, uint16_t *pre) {
    int run = 0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int m = lane + 64 * k;
        const uint64_t bal = __ballot(sel[k]);
        const int before = run + static_cast<int>(__builtin_amdgcn_mbcnt_hi(
                                     static_cast<uint32_t>(bal >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(bal), 0u)));
        if (m < n) pre[m] = static_cast<uint16_t>(before);
        if (sel[k]) {
            oeta[before] = eta[k];
            ophi[before] = phi[k];
        }
        run += __popcll(bal);
    }
    if (lane == 0) pre[n] = static_cast<uint16_t>(run);
}

// Six wavefronts per SIMD (at most 80 VGPRs): measured the best trade
// between latency hiding and the registers that hold a tile in flight.
template <typename T, bool EXT, int WAVES, int EVPL, bool LDSH>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(6))) void pipeline_kernel(PipeArgs P) {
    using C = Caps<EVPL, EXT>;
    constexpr int TW = C::TW, JK = C::JK, MK = C::MK, EK = C::EK;
    __shared__ WaveLds<EVPL, EXT> wl[WAVES];
    extern __shared__ double dyn[];  // [sumw | counts (u32) | edges] per workgroup

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    auto &L = wl[wave];

    double *sw_s = dyn;
    uint32_t *c_s = reinterpret_cast<uint32_t *>(dyn + (LDSH ? P.ds_slots : 0));
    float *e_s = reinterpret_cast<float *>(c_s + (LDSH ? P.ds_slots : 0));
    if (LDSH) {
        for (int i = tid; i < P.ds_slots; i += 64 * WAVES) {
            sw_s[i] = 0.0;
            c_s[i] = 0u;
        }
    }
    const float *edges = P.edges;
    if (P.edges_in_lds) {
        for (int i = tid; i < P.n_edges; i += 64 * WAVES) e_s[i] = as_const(P.edges)[i];
        edges = e_s;
    }
    __syncthreads();

    for (int ci = P.chunk_begin + blockIdx.x; ci < P.chunk_end; ci += gridDim.x) {
        const Chunk CH = as_const(P.chunks)[ci];
        const auto &D = as_const(P.ds)[CH.d];  // read in place, like the query table
        HistSink<LDSH> sink;
        if (LDSH) {
            sink.sw = sw_s;
            sink.c32 = c_s;
        } else {
            sink.sw = P.sumw + D.hist0;
            sink.c64 = P.counts + D.hist0;
        }
        const bool has_iso = D.miso != nullptr;
        const bool has_el = EXT && D.eoff != nullptr;
        const bool has_bt = EXT && D.jbt != nullptr;

        // tile bounds are fetched one tile ahead (scalar loads that overlap
        // the current tile's vector loads)
        int64_t t = CH.t0 + wave;
        TileBounds nb{};
        if (t < CH.t1) {
            const int64_t e0 = t * TW;
            nb = tile_bounds<EXT>(D, has_el, e0, static_cast<int>(min<int64_t>(TW, D.n_events - e0)));
        }
        for (; t < CH.t1; t += WAVES) {
            const int64_t e0 = t * TW;
            const int ne = static_cast<int>(min<int64_t>(TW, D.n_events - e0));
            const TileBounds B = nb;
            if (t + WAVES < CH.t1) {
                const int64_t e1 = (t + WAVES) * TW;
                nb = tile_bounds<EXT>(D, has_el, e1, static_cast<int>(min<int64_t>(TW, D.n_events - e1)));
            }
            if (B.J1 - B.J0 > C::JC || B.M1 - B.M0 > C::MC || B.L1 - B.L0 > C::EC) {
                const DsDev Dc = D;
#pragma unroll
                for (int r = 0; r < EVPL; ++r) {
                    const int ev = lane + 64 * r;
                    if (ev < ne) event_direct<T, EXT, LDSH>(P, Dc, e0 + ev, edges, sink);
                }
                continue;
            }
            const int nj = static_cast<int>(B.J1 - B.J0), nm = static_cast<int>(B.M1 - B.M0);
            const int nl = static_cast<int>(B.L1 - B.L0);

            // ---- 1. all of the tile's loads in flight at once: both offsets of
            // each event lane's event (tile-relative), its weight, and up to JK
            // jets, MK muons and EK electrons per lane
            // tile-base pointers (scalar) and 32-bit lane offsets
            const int64_t *jo = D.joff + e0, *mo = D.moff + e0, *lo = has_el ? D.eoff + e0 : nullptr;
            const float *wp = D.w ? D.w + e0 : nullptr;
            const T *cjpt = static_cast<const T *>(D.jpt) + B.J0, *cjeta = static_cast<const T *>(D.jeta) + B.J0;
            const T *cjphi = static_cast<const T *>(D.jphi) + B.J0;
            const T *cjbt = has_bt ? static_cast<const T *>(D.jbt) + B.J0 : nullptr;
            const T *cmpt = static_cast<const T *>(D.mpt) + B.M0, *cmeta = static_cast<const T *>(D.meta) + B.M0;
            const T *cmphi = static_cast<const T *>(D.mphi) + B.M0;
            const T *cmiso = has_iso ? static_cast<const T *>(D.miso) + B.M0 : nullptr;
            int32_t jb[EVPL], je[EVPL], mb[EVPL], me[EVPL], lb[EVPL], le[EVPL];
            float wv[EVPL];
#pragma unroll
            for (int r = 0; r < EVPL; ++r) {
                const int ev = lane + 64 * r;
                jb[r] = je[r] = mb[r] = me[r] = lb[r] = le[r] = 0;
                wv[r] = 1.0f;
                if (ev < ne) {
                    jb[r] = static_cast<int32_t>(jo[ev] - B.J0);
                    je[r] = static_cast<int32_t>(jo[ev + 1] - B.J0);
                    mb[r] = static_cast<int32_t>(mo[ev] - B.M0);
                    me[r] = static_cast<int32_t>(mo[ev + 1] - B.M0);
                    if (EXT && has_el) {
                        lb[r] = static_cast<int32_t>(lo[ev] - B.L0);
                        le[r] = static_cast<int32_t>(lo[ev + 1] - B.L0);
                    }
                    if (wp) wv[r] = wp[ev];
                }
            }
            float jpt[JK] = {}, jeta[JK] = {}, jphi[JK] = {}, jbt[EXT ? JK : 1] = {};
#pragma unroll
            for (int k = 0; k < JK; ++k) {
                const int j = lane + 64 * k;
                if (j < nj) {
                    jpt[k] = ldf(cjpt, j);
                    jeta[k] = ldf(cjeta, j);
                    jphi[k] = ldf(cjphi, j);
                    if (EXT && has_bt) jbt[EXT ? k : 0] = ldf(cjbt, j);
                }
            }
            float mpt[MK] = {}, meta[MK] = {}, mphi[MK] = {}, miso[MK] = {};
#pragma unroll
            for (int k = 0; k < MK; ++k) {
                const int m = lane + 64 * k;
                if (m < nm) {
                    mpt[k] = ldf(cmpt, m);
                    meta[k] = ldf(cmeta, m);
                    mphi[k] = ldf(cmphi, m);
                    if (has_iso) miso[k] = ldf(cmiso, m);
                }
            }
            float lpt[EK] = {}, leta[EK] = {}, lphi[EK] = {};
            if (EXT && has_el) {
                const T *cept = static_cast<const T *>(D.ept) + B.L0, *ceeta = static_cast<const T *>(D.eeta) + B.L0;
                const T *cephi = static_cast<const T *>(D.ephi) + B.L0;
#pragma unroll
                for (int k = 0; k < EK; ++k) {
                    const int m = lane + 64 * k;
                    if (m < nl) {
                        lpt[k] = ldf(cept, m);
                        leta[k] = ldf(ceeta, m);
                        lphi[k] = ldf(cephi, m);
                    }
                }
            }
            // Every value above is used here, so the compiler issues all of the
            // tile's loads before this point and waits once, instead of sinking
            // each load to its first use (one HBM round trip per tile).
#pragma unroll
            for (int r = 0; r < EVPL; ++r)
                asm volatile("" ::"v"(jb[r]), "v"(je[r]), "v"(mb[r]), "v"(me[r]), "v"(wv[r]));
#pragma unroll
            for (int k = 0; k < JK; ++k) asm volatile("" ::"v"(jpt[k]), "v"(jeta[k]), "v"(jphi[k]));
#pragma unroll
            for (int k = 0; k < MK; ++k) asm volatile("" ::"v"(mpt[k]), "v"(meta[k]), "v"(mphi[k]), "v"(miso[k]));
            if (EXT) {
#pragma unroll
                for (int r = 0; r < EVPL; ++r) asm volatile("" ::"v"(lb[r]), "v"(le[r]));
#pragma unroll
                for (int k = 0; k < JK; ++k) asm volatile("" ::"v"(jbt[EXT ? k : 0]));
#pragma unroll
                for (int k = 0; k < EK; ++k) asm volatile("" ::"v"(lpt[k]), "v"(leta[k]), "v"(lphi[k]));
            }

            for (int q = 0; q < P.n_q; ++q) {
                // the query's fields are read in place (scalar loads near their
                // uses) rather than copied: a copy would hold ~45 SGPRs for the
                // whole query and spill
                const auto &Q = as_const(P.qs)[q];
                if (!Q.active) continue;
                // ---- 2. lepton selection; selected leptons compacted into LDS
                {
                    bool sel[MK];
#pragma unroll
                    for (int k = 0; k < MK; ++k)
                        sel[k] = (lane + 64 * k < nm) && mpt[k] > Q.mu_pt && fabsf(meta[k]) < Q.mu_abseta &&
                                 (!has_iso || miso[k] < Q.mu_iso);
                    compact<MK>(sel, meta, mphi, nm, lane, L.seta, L.sphi, L.mpre);
                }
                if (EXT) {
                    bool sel[EK];
#pragma unroll
                    for (int k = 0; k < EK; ++k)
                        sel[k] = (lane + 64 * k < nl) && lpt[k] > Q.el_pt && fabsf(leta[k]) < Q.el_abseta;
                    compact<EK>(sel, leta, lphi, nl, lane, L.sea, L.sep, L.epre);
                }
                wave_sync();
                // ---- 3. each event lane writes its selected-lepton range over its jets
                int nmu[EVPL];
#pragma unroll
                for (int r = 0; r < EVPL; ++r) {
                    nmu[r] = 0;
                    const int ev = lane + 64 * r;
                    if (ev < ne) {
                        const int s0 = L.mpre[mb[r]];
                        nmu[r] = L.mpre[me[r]] - s0;
                        const uint32_t pk = static_cast<uint32_t>(s0) | (static_cast<uint32_t>(nmu[r]) << 16);
                        uint32_t pke = 0;
                        if (EXT) {
                            const int u0 = L.epre[lb[r]];
                            pke = static_cast<uint32_t>(u0) | (static_cast<uint32_t>(L.epre[le[r]] - u0) << 16);
                        }
                        for (int k = jb[r]; k < je[r]; ++k) {
                            L.jr[k].rng = pk;
                            if (EXT) L.jre[k] = pke;
                        }
                    }
                }
                wave_sync();
                // ---- 4. cone test per jet against its event's selected leptons
#pragma unroll
                for (int k = 0; k < JK; ++k) {
                    const int j = lane + 64 * k;
                    if (j < nj) {
                        const uint32_t pk = L.jr[j].rng;
                        const int c0 = static_cast<int>(pk & 0xffffu), c1 = c0 + static_cast<int>(pk >> 16);
                        bool hit = false;
                        int i = c0;
                        // two leptons per step: both LDS reads in flight before the math
                        for (; i + 2 <= c1; i += 2) {
                            const float e0 = L.seta[i], p0 = L.sphi[i], e1 = L.seta[i + 1], p1 = L.sphi[i + 1];
                            hit |= delta_r2(jeta[k], jphi[k], e0, p0) <= Q.thr2;
                            hit |= delta_r2(jeta[k], jphi[k], e1, p1) <= Q.thr2;
                        }
                        if (i < c1) hit |= delta_r2(jeta[k], jphi[k], L.seta[i], L.sphi[i]) <= Q.thr2;
                        if (EXT) {
                            const uint32_t pe = L.jre[j];
                            const int u0 = static_cast<int>(pe & 0xffffu), u1 = u0 + static_cast<int>(pe >> 16);
                            for (int i = u0; i < u1; ++i) hit |= delta_r2(jeta[k], jphi[k], L.sea[i], L.sep[i]) <= Q.thr2;
                        }
                        const bool ok = !hit && fabsf(jeta[k]) < Q.jet_abseta;
                        L.jr[j].pt = ok ? jpt[k] : __builtin_nanf("");
                        if (EXT) L.bt[j] = (has_bt && jbt[EXT ? k : 0] > Q.btag) ? 1 : 0;
                    }
                }
                wave_sync();
                // ---- 5. per-event reductions, event cut, fills
                // Walk an event's jets in order for one scale s: left-to-right
                // float32 H_T over the selected ones, their count and maximum.
                // Branch-free, two jets per step (both LDS reads in flight);
                // adding only selected x keeps the sum order of the definition,
                // and the maximum is updated on a strict '>', which keeps the
                // first of equal values, as the definition does.
                auto walk = [&](int j0, int j1, float s, float &ht, float &lead, int &njs, int &nbt) {
                    njs = 0;
                    nbt = 0;
                    ht = 0.0f;
                    lead = -INFINITY;
                    auto step = [&](float x, int k) {
                        const bool sel = x > Q.jet_pt;
                        const float hs = ht + x;
                        ht = sel ? hs : ht;
                        lead = (sel && x > lead) ? x : lead;
                        njs += sel ? 1 : 0;
                        if (EXT) nbt += sel ? L.bt[k] : 0;
                    };
                    int k = j0;
                    for (; k + 2 <= j1; k += 2) {
                        const float x0 = L.jr[k].pt * s, x1 = L.jr[k + 1].pt * s;
                        step(x0, k);
                        step(x1, k + 1);
                    }
                    if (k < j1) step(L.jr[k].pt * s, k);
                };
                auto fill = [&](int v, float ht, float lead, int njs, double w) {
                    // separate calls so each knows its address space (LDS or
                    // global) and reads the edges without flat loads
                    if (P.edges_in_lds)
                        fill3(sink, Q, e_s, v, ht, lead, njs, w);
                    else
                        fill3(sink, Q, P.edges, v, ht, lead, njs, w);
                };
                if (Q.n_scale == 1) {
                    const float s = as_const(P.scales)[Q.scale0];
#pragma unroll
                    for (int r = 0; r < EVPL; ++r) {
                        const int ev = lane + 64 * r;
                        if (ev < ne) {
                            float ht, lead;
                            int njs, nbt;
                            walk(jb[r], je[r], s, ht, lead, njs, nbt);
                            if (nmu[r] >= Q.min_mu && njs >= Q.min_jet && (!has_bt || nbt >= Q.min_b))
                                fill(0, ht, lead, njs, static_cast<double>(wv[r]));
                        }
                    }
                } else {
                    // Several scales: lanes take (event, scale) pairs, event-major,
                    // so one round covers a few events (shorter divergent walks)
                    // and its fills spread over different histograms.
#pragma unroll
                    for (int r = 0; r < EVPL; ++r) {
                        const int ev = lane + 64 * r;
                        if (ev < ne) {
                            L.evjr[ev] = static_cast<uint32_t>(jb[r]) | (static_cast<uint32_t>(je[r]) << 16);
                            L.evnmu[ev] = static_cast<uint16_t>(nmu[r]);
                            L.evw[ev] = wv[r];
                        }
                    }
                    wave_sync();
                    const int V = Q.n_scale;
                    const int npairs = ne * V;
                    int e = lane / V, v = lane - (lane / V) * V;
                    const int de = 64 / V, dv = 64 - (64 / V) * V;
                    for (int i = lane; i < npairs; i += 64) {
                        const uint32_t jr = L.evjr[e];
                        float ht, lead;
                        int njs, nbt;
                        walk(static_cast<int>(jr & 0xffffu), static_cast<int>(jr >> 16), P.scales[Q.scale0 + v], ht,
                             lead, njs, nbt);
                        if (L.evnmu[e] >= Q.min_mu && njs >= Q.min_jet && (!has_bt || nbt >= Q.min_b))
                            fill(v, ht, lead, njs, static_cast<double>(L.evw[e]));
                        e += de;
                        v += dv;
                        if (v >= V) {
                            v -= V;
                            e += 1;
                        }
                    }
                }
                wave_sync();
            }
        }
        // merge the LDS histograms when the next chunk is another dataset (or none)
        if (LDSH) {
            const int nci = ci + static_cast<int>(gridDim.x);
            if (nci >= P.chunk_end || as_const(P.chunks)[nci].d != CH.d) {
                __syncthreads();
                for (int q = 0; q < P.n_q; ++q) {
                    const QDev Q = as_const(P.qs)[q];
                    if (!Q.active) continue;
                    for (int v = 0; v < Q.n_scale; ++v)
                        for (int h = 0; h < 3; ++h) {
                            const int ls = Q.lslot0 + v * Q.lper_scale + Q.lhoff[h];
                            const int64_t gs = D.hist0 + Q.gslot0 + v * Q.gper_scale + Q.ghoff[h];
                            for (int i = tid; i < Q.nbins[h] + 2; i += 64 * WAVES) {
                                const uint32_t c = c_s[ls + i];
                                if (c) {
                                    atomic_add_u64(&P.counts[gs + i], c);
                                    atomic_add_f64(&P.sumw[gs + i], sw_s[ls + i]);
                                    c_s[ls + i] = 0u;
                                    sw_s[ls + i] = 0.0;
                                }
                            }
                        }
                }
                __syncthreads();
            }
        }
    }
}

using KernelFn = void (*)(PipeArgs);

template <typename T, bool EXT, int WAVES, int EVPL, bool LDSH>
static KernelFn kfn() {
    return reinterpret_cast<KernelFn>(&pipeline_kernel<T, EXT, WAVES, EVPL, LDSH>);
}

template <typename T, bool EXT, int WAVES, int EVPL>
static KernelFn pick_h(bool ldsh) {
    return ldsh ? kfn<T, EXT, WAVES, EVPL, true>() : kfn<T, EXT, WAVES, EVPL, false>();
}

template <typename T, bool EXT>
static KernelFn pick_shape(int block, int evpt, bool ldsh) {
    if (block == 512) return evpt == 2 ? pick_h<T, EXT, 8, 2>(ldsh) : pick_h<T, EXT, 8, 1>(ldsh);
    return evpt == 2 ? pick_h<T, EXT, 4, 2>(ldsh) : pick_h<T, EXT, 4, 1>(ldsh);
}

static KernelFn pick_kernel(int dtype, bool ext, int block, int evpt, bool ldsh) {
    if (dtype == HEPK_F16) return ext ? pick_shape<_Float16, true>(block, evpt, ldsh)
                                      : pick_shape<_Float16, false>(block, evpt, ldsh);
    return ext ? pick_shape<float, true>(block, evpt, ldsh) : pick_shape<float, false>(block, evpt, ldsh);
}

// LDS for the workgroup's private histograms: up to 64 KiB (60 histograms of
// 100 bins fit); larger sets go to global atomics.  More LDS lowers occupancy,
// which the launch-configuration search weighs against atomic contention.
constexpr int kMaxLdsHistBytes = 64 * 1024;
constexpr int kMaxLdsEdgeBytes = 4 * 1024;

}  // namespace hepk

struct hepk_plan_s {
    int device = 0;
    int32_t n_ds = 0, n_q = 0;
    int dtype = HEPK_F32;
    bool ext = false;
    bool shared = false;
    hepk_tune tune{};
    int grid = 0;
    hepk::KernelFn fn_lds = nullptr, fn_glob = nullptr;
    hepk::PipeArgs args{};             // table pointers; chunk range and histograms set per launch
    int32_t n_chunks_all = 0;          // balanced chunks of the full pass: [0, n_chunks_all)
    std::vector<int32_t> full_begin;   // n_ds + 1: first chunk of each dataset in the full list
    std::vector<int32_t> own_begin;    // n_ds + 1: each dataset's own balanced chunk list
    int64_t ds_block = 0;              // histogram slots per dataset block
    int64_t n_slots = 0;
    std::vector<hepk::QDev> qd;        // host copy of the query table
    std::vector<int32_t> cap_bins;     // (slot, h): reserved bins
    std::vector<int32_t> cap_scales;   // slot: reserved scales
    int32_t lds_slots = 0;             // LDS histogram slots of the active queries
    int32_t n_edges = 0;
    bool edges_lds = false;
    void *dev_mem = nullptr;
    hepk::QDev *d_q = nullptr;
    float *d_scales = nullptr, *d_edges = nullptr;
    // pinned staging ring for hepk_plan_set_query
    char *pinned = nullptr;
    size_t stage_bytes = 0;
    int ring_pos = 0;
    std::vector<hipEvent_t> ring_ev;
    std::vector<bool> ring_used;
    // graph launch
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipGraphNode_t gnode = nullptr;
    hepk::KernelFn gfn = nullptr;
    hepk::PipeArgs gargs{};
    size_t glds = 0;
    int ggrid = 0;
};

namespace hepk {

constexpr int kStageRing = 32;

// LDS layout of the active queries (compact) and whether it fits in LDS.
static void relayout(hepk_plan p) {
    int32_t acc = 0;
    for (auto &o : p->qd) {
        o.lslot0 = acc;
        int32_t per = 0;
        for (int h = 0; h < 3; ++h) {
            o.lhoff[h] = per;
            per += o.nbins[h] + 2;
        }
        o.lper_scale = per;
        if (o.active) acc += per * o.n_scale;
    }
    p->lds_slots = acc;
}

static bool use_lds_hist(hepk_plan p) {
    return p->tune.hist_mode == 0 &&
           static_cast<size_t>(p->lds_slots) * (sizeof(double) + sizeof(uint32_t)) <= static_cast<size_t>(kMaxLdsHistBytes);
}

// Fills the query-dependent fields of a table entry; the caller has checked q.
static void set_qdev(QDev &o, const hepk_query &Q, const float *const edges[3]) {
    o.mu_pt = Q.mu_pt;
    o.mu_abseta = Q.mu_abseta;
    o.mu_iso = Q.mu_iso;
    o.el_pt = Q.el_pt;
    o.el_abseta = Q.el_abseta;
    o.jet_pt = Q.jet_pt;
    o.jet_abseta = Q.jet_abseta;
    o.thr2 = Q.dr * Q.dr;  // rounded once to float32
    o.btag = Q.btag;
    o.min_mu = Q.min_mu;
    o.min_jet = Q.min_jet;
    o.min_b = Q.min_b;
    o.n_scale = Q.n_scale;
    o.active = 1;
    for (int h = 0; h < 3; ++h) {
        const int nb = Q.nbins[h];
        const float *e = edges[h];
        o.nbins[h] = nb;
        const float span = e[nb] - e[0];
        o.lo[h] = e[0];
        o.hi[h] = e[nb];
        o.inv_w[h] = (span > 0.0f && std::isfinite(span)) ? static_cast<float>(nb) / span : 0.0f;
    }
}

static int check_query(const hepk_query &Q, int i) {
    HEPK_REQUIRE(Q.n_scale >= 1 && Q.scales, "query %d needs >= 1 scale", i);
    for (int h = 0; h < 3; ++h) {
        HEPK_REQUIRE(Q.nbins[h] >= 1 && Q.edges[h], "query %d histogram %d invalid", i, h);
        for (int k = 0; k < Q.nbins[h]; ++k)
            HEPK_REQUIRE(Q.edges[h][k] < Q.edges[h][k + 1], "query %d edges %d not strictly increasing at %d", i,
                         h, k);
    }
    return HEPK_OK;
}

static int64_t hist_base(hepk_plan p, int d) { return p->shared ? 0 : d * p->ds_block; }

struct Launch {
    KernelFn fn;
    int grid, block;
    size_t lds;
    PipeArgs a;
};

static Launch make_launch(hepk_plan p, int32_t c0, int32_t c1, double *sumw, uint64_t *counts) {
    Launch L{};
    const bool ldsh = use_lds_hist(p);
    L.fn = ldsh ? p->fn_lds : p->fn_glob;
    L.block = p->tune.block;
    L.grid = std::max(1, std::min(p->grid, c1 - c0));
    L.lds = (ldsh ? static_cast<size_t>(p->lds_slots) * (sizeof(double) + sizeof(uint32_t)) : 0) +
            (p->edges_lds ? static_cast<size_t>(p->n_edges) * sizeof(float) : 0);
    L.a = p->args;
    L.a.chunk_begin = c0;
    L.a.chunk_end = c1;
    L.a.ds_slots = ldsh ? p->lds_slots : 0;
    L.a.sumw = sumw;
    L.a.counts = counts;
    return L;
}

static int run_launch(const Launch &L, hipStream_t stream) {
    void *kargs[] = {const_cast<PipeArgs *>(&L.a)};
    HEPK_HIP(hipLaunchKernel(reinterpret_cast<const void *>(L.fn), dim3(L.grid), dim3(L.block), kargs, L.lds,
                             stream));
    return check_launch("hepk_pipeline");
}

static bool any_active(hepk_plan p) {
    for (const auto &o : p->qd)
        if (o.active) return true;
    return false;
}

static void free_plan(hepk_plan p) {
    if (!p) return;
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    for (auto e : p->ring_ev) (void)hipEventDestroy(e);
    if (p->pinned) (void)hipHostFree(p->pinned);
    if (p->dev_mem) (void)hipFree(p->dev_mem);
    delete p;
}

}  // namespace hepk

static int plan_fail(hepk_plan p, int rc) {
    hepk::free_plan(p);
    return rc;
}

extern "C" int hepk_plan_create_ex(const hepk_dataset *ds, int32_t n_ds, const hepk_query *q, int32_t n_query,
                                   const hepk_plan_opts *opts, hepk_plan *out) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(out, "hepk_plan_create: out is NULL");
    *out = nullptr;
    HEPK_REQUIRE(n_ds >= 1 && ds, "hepk_plan_create: need at least one dataset");
    HEPK_REQUIRE(n_query >= 1 && q, "hepk_plan_create: need at least one query");
    const int dtype = ds[0].dtype;
    HEPK_REQUIRE(dtype == HEPK_F32 || dtype == HEPK_F16, "hepk_plan_create: content dtype %d unsupported", dtype);
    bool ext = false;
    for (int d = 0; d < n_ds; ++d) {
        const hepk_dataset &D = ds[d];
        HEPK_REQUIRE(D.dtype == dtype, "hepk_plan_create: dataset %d dtype differs from dataset 0", d);
        HEPK_REQUIRE(D.n_events >= 0 && D.n_events < (int64_t(1) << 31),
                     "hepk_plan_create: dataset %d n_events %lld out of [0, 2^31)", d, (long long)D.n_events);
        HEPK_REQUIRE(D.jets.offsets && D.muons.offsets, "hepk_plan_create: dataset %d lacks jet/muon offsets", d);
        // an empty dataset never touches its content columns
        const bool any = D.n_events > 0;
        HEPK_REQUIRE(!any || (D.jets.pt && D.jets.eta && D.jets.phi), "hepk_plan_create: dataset %d jet column NULL",
                     d);
        HEPK_REQUIRE(!any || (D.muons.pt && D.muons.eta && D.muons.phi),
                     "hepk_plan_create: dataset %d muon column NULL", d);
        if (D.electrons.offsets) {
            HEPK_REQUIRE(!any || (D.electrons.pt && D.electrons.eta && D.electrons.phi),
                         "hepk_plan_create: dataset %d electron column NULL", d);
            ext = true;
        }
        if (D.jets.extra) ext = true;
    }
    for (int i = 0; i < n_query; ++i) {
        int rc = check_query(q[i], i);
        if (rc) return rc;
    }
    hepk_plan_opts o{};
    if (opts) o = *opts;
    hepk_tune t = o.tune;
    if (t.block == 0) t = hepk_tune{512, 1, 0, 0};
    HEPK_REQUIRE(t.block == 256 || t.block == 512, "hepk_plan_create: block %d not 256 or 512", t.block);
    HEPK_REQUIRE(t.ev_per_thread == 1 || t.ev_per_thread == 2, "hepk_plan_create: ev_per_thread %d not 1 or 2",
                 t.ev_per_thread);
    HEPK_REQUIRE(t.hist_mode == 0 || t.hist_mode == 1, "hepk_plan_create: hist_mode %d not 0 or 1", t.hist_mode);
    HEPK_REQUIRE(t.grid >= 0, "hepk_plan_create: grid < 0");
    HEPK_REQUIRE(o.reserve_bins >= 0 && o.reserve_bins < (1 << 20), "hepk_plan_create: reserve_bins out of range");

    hepk_plan p = new hepk_plan_s();
    if (hipGetDevice(&p->device) != hipSuccess) {
        set_error("hepk_plan_create: no current HIP device");
        return plan_fail(p, HEPK_EHIP);
    }
    p->n_ds = n_ds;
    p->n_q = n_query;
    p->dtype = dtype;
    p->ext = ext;
    p->shared = o.shared_hist != 0;

    // query slots: reserved bins/scales, global histogram blocks, edge and scale regions
    p->qd.assign(n_query, QDev{});
    p->cap_bins.assign(3 * n_query, 0);
    p->cap_scales.assign(n_query, 0);
    std::vector<float> edge_table, scales;
    int64_t gacc = 0;
    int32_t max_cap = 0, max_sc = 0;
    for (int i = 0; i < n_query; ++i) {
        QDev &e = p->qd[i];
        set_qdev(e, q[i], q[i].edges);
        p->cap_scales[i] = q[i].n_scale;
        max_sc = std::max(max_sc, q[i].n_scale);
        e.scale0 = static_cast<int32_t>(scales.size());
        for (int v = 0; v < q[i].n_scale; ++v) scales.push_back(q[i].scales[v]);
        int32_t per = 0;
        for (int h = 0; h < 3; ++h) {
            const int cap = std::max(q[i].nbins[h], o.reserve_bins);
            p->cap_bins[3 * i + h] = cap;
            max_cap = std::max(max_cap, cap);
            e.ghoff[h] = per;
            per += cap + 2;
            e.ebase[h] = static_cast<int32_t>(edge_table.size());
            edge_table.insert(edge_table.end(), q[i].edges[h], q[i].edges[h] + q[i].nbins[h] + 1);
            edge_table.resize(e.ebase[h] + cap + 1, 0.0f);
        }
        e.gper_scale = per;
        e.gslot0 = static_cast<int32_t>(gacc);
        gacc += static_cast<int64_t>(per) * q[i].n_scale;
    }
    if (gacc >= (int64_t(1) << 30) || edge_table.size() >= (size_t(1) << 30)) {
        set_error("hepk_plan_create: %lld histogram slots per dataset is too many", (long long)gacc);
        return plan_fail(p, HEPK_EINVAL);
    }
    p->ds_block = gacc;
    p->n_slots = p->shared ? gacc : gacc * n_ds;
    p->n_edges = static_cast<int32_t>(edge_table.size());
    p->edges_lds = static_cast<size_t>(p->n_edges) * sizeof(float) <= static_cast<size_t>(kMaxLdsEdgeBytes);
    p->tune = t;
    relayout(p);

    const int waves = t.block / 64;
    const int tw = 64 * t.ev_per_thread;
    std::vector<DsDev> dd(n_ds);
    std::vector<int64_t> tiles(n_ds);
    int64_t total_tiles = 0;
    for (int d = 0; d < n_ds; ++d) {
        const hepk_dataset &D = ds[d];
        DsDev &e = dd[d];
        e.n_events = D.n_events;
        e.joff = D.jets.offsets;
        e.moff = D.muons.offsets;
        e.eoff = D.electrons.offsets;
        e.jpt = D.jets.pt;
        e.jeta = D.jets.eta;
        e.jphi = D.jets.phi;
        e.jbt = D.jets.extra;
        e.mpt = D.muons.pt;
        e.meta = D.muons.eta;
        e.mphi = D.muons.phi;
        e.miso = D.muons.extra;
        e.ept = D.electrons.pt;
        e.eeta = D.electrons.eta;
        e.ephi = D.electrons.phi;
        e.w = D.weights;
        e.hist0 = hist_base(p, d);
        tiles[d] = ceil_div(D.n_events, tw);
        total_tiles += tiles[d];
    }

    p->fn_lds = pick_kernel(dtype, ext, t.block, t.ev_per_thread, true);
    p->fn_glob = pick_kernel(dtype, ext, t.block, t.ev_per_thread, false);
    const size_t lds_hist = use_lds_hist(p) ? static_cast<size_t>(p->lds_slots) * 12 : 0;
    const size_t lds_bytes = lds_hist + (p->edges_lds ? p->n_edges * sizeof(float) : 0);
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(use_lds_hist(p) ? p->fn_lds : p->fn_glob), t.block,
            lds_bytes) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    int64_t grid = t.grid > 0 ? t.grid : static_cast<int64_t>(per_cu) * device_cus();

    // Work chunks: runs of tiles of one dataset, a multiple of the
    // wavefronts per workgroup long.  The full pass uses chunks of about
    // total/grid tiles (one per workgroup, plus those split at dataset ends);
    // each dataset also has its own list of about tiles/grid-sized chunks so
    // that a pass over that dataset alone fills the device.
    auto chunk_len = [&](int64_t n) {
        return std::max<int64_t>(waves, ceil_div(ceil_div(n, std::max<int64_t>(1, grid)), waves) * waves);
    };
    std::vector<Chunk> chunks;
    const int64_t per_all = chunk_len(total_tiles);
    p->full_begin.assign(n_ds + 1, 0);
    for (int d = 0; d < n_ds; ++d) {
        p->full_begin[d] = static_cast<int32_t>(chunks.size());
        for (int64_t t0 = 0; t0 < tiles[d]; t0 += per_all)
            chunks.push_back(Chunk{d, 0, t0, std::min(tiles[d], t0 + per_all)});
    }
    p->full_begin[n_ds] = static_cast<int32_t>(chunks.size());
    p->n_chunks_all = static_cast<int32_t>(chunks.size());
    p->own_begin.assign(n_ds + 1, 0);
    for (int d = 0; d < n_ds; ++d) {
        p->own_begin[d] = static_cast<int32_t>(chunks.size());
        const int64_t per = chunk_len(tiles[d]);
        for (int64_t t0 = 0; t0 < tiles[d]; t0 += per) chunks.push_back(Chunk{d, 0, t0, std::min(tiles[d], t0 + per)});
    }
    p->own_begin[n_ds] = static_cast<int32_t>(chunks.size());
    if (chunks.size() >= (size_t(1) << 31)) {
        set_error("hepk_plan_create: too many work chunks");
        return plan_fail(p, HEPK_EINVAL);
    }
    p->grid = static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(grid, std::max(1, p->n_chunks_all))));
    p->tune.grid = p->grid;

    // one device allocation for the tables
    const size_t sz_ds = sizeof(DsDev) * n_ds, sz_ch = sizeof(Chunk) * std::max<size_t>(1, chunks.size());
    const size_t sz_q = sizeof(QDev) * n_query, sz_sc = sizeof(float) * scales.size();
    const size_t sz_e = sizeof(float) * edge_table.size();
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t o_ds = 0, o_ch = al(sz_ds), o_q = o_ch + al(sz_ch), o_sc = o_q + al(sz_q), o_e = o_sc + al(sz_sc);
    const size_t total = o_e + al(sz_e);
    if (hipMalloc(&p->dev_mem, total) != hipSuccess) {
        set_error("hepk_plan_create: hipMalloc of %zu bytes failed", total);
        return plan_fail(p, HEPK_ENOMEM);
    }
    char *base = static_cast<char *>(p->dev_mem);
    std::vector<char> host(total, 0);
    std::memcpy(host.data() + o_ds, dd.data(), sz_ds);
    if (!chunks.empty()) std::memcpy(host.data() + o_ch, chunks.data(), sizeof(Chunk) * chunks.size());
    std::memcpy(host.data() + o_q, p->qd.data(), sz_q);
    if (sz_sc) std::memcpy(host.data() + o_sc, scales.data(), sz_sc);
    if (sz_e) std::memcpy(host.data() + o_e, edge_table.data(), sz_e);
    if (hipMemcpy(base, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
        set_error("hepk_plan_create: table upload failed");
        return plan_fail(p, HEPK_EHIP);
    }
    p->d_q = reinterpret_cast<QDev *>(base + o_q);
    p->d_scales = reinterpret_cast<float *>(base + o_sc);
    p->d_edges = reinterpret_cast<float *>(base + o_e);

    // staging ring: a full query table plus one slot's edges and scales per entry
    p->stage_bytes = al(sz_q) + al(sizeof(float) * 3 * (max_cap + 1)) + al(sizeof(float) * max_sc);
    if (hipHostMalloc(reinterpret_cast<void **>(&p->pinned), p->stage_bytes * kStageRing, hipHostMallocDefault) !=
        hipSuccess) {
        set_error("hepk_plan_create: pinned staging allocation failed");
        return plan_fail(p, HEPK_ENOMEM);
    }
    p->ring_ev.assign(kStageRing, nullptr);
    p->ring_used.assign(kStageRing, false);
    for (int r = 0; r < kStageRing; ++r)
        if (hipEventCreateWithFlags(&p->ring_ev[r], hipEventDisableTiming) != hipSuccess) {
            set_error("hepk_plan_create: event creation failed");
            return plan_fail(p, HEPK_EHIP);
        }

    PipeArgs &A = p->args;
    A.ds = reinterpret_cast<const DsDev *>(base + o_ds);
    A.qs = p->d_q;
    A.scales = p->d_scales;
    A.chunks = reinterpret_cast<const Chunk *>(base + o_ch);
    A.edges = p->d_edges;
    A.n_q = n_query;
    A.n_edges = p->n_edges;
    A.edges_in_lds = p->edges_lds ? 1 : 0;
    *out = p;
    return HEPK_OK;
}

extern "C" int hepk_plan_create(const hepk_dataset *ds, int32_t n_ds, const hepk_query *q, int32_t n_query,
                                const hepk_tune *tune, hepk_plan *out) {
    hepk_plan_opts o{};
    if (tune) o.tune = *tune;
    if (tune && tune->block == 0) {
        hepk::set_error("hepk_plan_create: block 0 not 256 or 512");
        return HEPK_EINVAL;
    }
    return hepk_plan_create_ex(ds, n_ds, q, n_query, &o, out);
}

extern "C" int hepk_plan_set_query(hepk_plan p, int32_t slot, const hepk_query *q, hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(p, "hepk_plan_set_query: plan is NULL");
    HEPK_REQUIRE(slot >= 0 && slot < p->n_q, "hepk_plan_set_query: slot %d out of [0, %d)", slot, p->n_q);
    if (q) {
        int rc = check_query(*q, slot);
        if (rc) return rc;
        HEPK_REQUIRE(q->n_scale <= p->cap_scales[slot], "hepk_plan_set_query: %d scales, slot holds %d", q->n_scale,
                     p->cap_scales[slot]);
        for (int h = 0; h < 3; ++h)
            HEPK_REQUIRE(q->nbins[h] <= p->cap_bins[3 * slot + h], "hepk_plan_set_query: %d bins, slot holds %d",
                         q->nbins[h], p->cap_bins[3 * slot + h]);
    }
    const int r = p->ring_pos;
    p->ring_pos = (p->ring_pos + 1) % kStageRing;
    if (p->ring_used[r]) HEPK_HIP(hipEventSynchronize(p->ring_ev[r]));
    char *st = p->pinned + r * p->stage_bytes;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t sz_q = sizeof(QDev) * p->n_q;
    QDev &e = p->qd[slot];
    const int max_cap = *std::max_element(p->cap_bins.begin(), p->cap_bins.end());
    float *st_e = reinterpret_cast<float *>(st + al(sz_q));
    float *st_s = reinterpret_cast<float *>(st + al(sz_q) + al(sizeof(float) * 3 * (max_cap + 1)));
    if (q) {
        set_qdev(e, *q, q->edges);
        for (int h = 0; h < 3; ++h) std::memcpy(st_e + h * (max_cap + 1), q->edges[h], sizeof(float) * (q->nbins[h] + 1));
        std::memcpy(st_s, q->scales, sizeof(float) * q->n_scale);
    } else {
        e.active = 0;
    }
    relayout(p);
    std::memcpy(st, p->qd.data(), sz_q);
    if (q) {
        for (int h = 0; h < 3; ++h)
            HEPK_HIP(hipMemcpyAsync(p->d_edges + e.ebase[h], st_e + h * (max_cap + 1), sizeof(float) * (q->nbins[h] + 1),
                                    hipMemcpyHostToDevice, stream));
        HEPK_HIP(hipMemcpyAsync(p->d_scales + e.scale0, st_s, sizeof(float) * q->n_scale, hipMemcpyHostToDevice,
                                stream));
    }
    HEPK_HIP(hipMemcpyAsync(p->d_q, st, sz_q, hipMemcpyHostToDevice, stream));
    HEPK_HIP(hipEventRecord(p->ring_ev[r], stream));
    p->ring_used[r] = true;
    return HEPK_OK;
}

extern "C" int hepk_plan_hist_slots(hepk_plan p, int64_t *n_slots) {
    hepk::clear_error();
    HEPK_REQUIRE(p && n_slots, "hepk_plan_hist_slots: NULL argument");
    *n_slots = p->n_slots;
    return HEPK_OK;
}

extern "C" int hepk_plan_hist_offset(hepk_plan p, int32_t d, int32_t iq, int32_t v, int32_t h, int64_t *offset,
                                     int32_t *nbins) {
    hepk::clear_error();
    HEPK_REQUIRE(p && offset && nbins, "hepk_plan_hist_offset: NULL argument");
    HEPK_REQUIRE(d >= 0 && d < p->n_ds && iq >= 0 && iq < p->n_q && h >= 0 && h < 3,
                 "hepk_plan_hist_offset: index out of range");
    const hepk::QDev &e = p->qd[iq];
    HEPK_REQUIRE(v >= 0 && v < p->cap_scales[iq], "hepk_plan_hist_offset: scale index out of range");
    *offset = hepk::hist_base(p, d) + e.gslot0 + static_cast<int64_t>(v) * e.gper_scale + e.ghoff[h];
    *nbins = e.nbins[h];
    return HEPK_OK;
}

extern "C" int hepk_plan_get_tune(hepk_plan p, hepk_tune *tune) {
    hepk::clear_error();
    HEPK_REQUIRE(p && tune, "hepk_plan_get_tune: NULL argument");
    *tune = p->tune;
    tune->hist_mode = hepk::use_lds_hist(p) ? 0 : 1;
    return HEPK_OK;
}

static int pipeline_chunks(hepk_plan p, int32_t c0, int32_t c1, double *sumw, uint64_t *counts, hipStream_t stream) {
    using namespace hepk;
    if (c1 <= c0 || !any_active(p)) return HEPK_OK;
    int dev = 0;
    HEPK_HIP(hipGetDevice(&dev));
    HEPK_REQUIRE(dev == p->device, "hepk_pipeline: plan made on device %d, current device %d", p->device, dev);
    return run_launch(make_launch(p, c0, c1, sumw, counts), stream);
}

extern "C" int hepk_pipeline(hepk_plan p, double *sumw, uint64_t *counts, hipStream_t stream) {
    hepk::clear_error();
    HEPK_REQUIRE(p, "hepk_pipeline: plan is NULL");
    HEPK_REQUIRE(sumw && counts, "hepk_pipeline: histogram buffers are NULL");
    return pipeline_chunks(p, 0, p->n_chunks_all, sumw, counts, stream);
}

extern "C" int hepk_pipeline_range(hepk_plan p, int32_t d0, int32_t nd, double *sumw, uint64_t *counts,
                                   hipStream_t stream) {
    hepk::clear_error();
    HEPK_REQUIRE(p, "hepk_pipeline_range: plan is NULL");
    HEPK_REQUIRE(sumw && counts, "hepk_pipeline_range: histogram buffers are NULL");
    HEPK_REQUIRE(d0 >= 0 && nd >= 0 && d0 + nd <= p->n_ds, "hepk_pipeline_range: datasets [%d, %d) out of [0, %d)",
                 d0, d0 + nd, p->n_ds);
    if (nd == 1) return pipeline_chunks(p, p->own_begin[d0], p->own_begin[d0 + 1], sumw, counts, stream);
    return pipeline_chunks(p, p->full_begin[d0], p->full_begin[d0 + nd], sumw, counts, stream);
}

extern "C" int hepk_pipeline_graph(hepk_plan p, double *sumw, uint64_t *counts, hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(p, "hepk_pipeline_graph: plan is NULL");
    HEPK_REQUIRE(sumw && counts, "hepk_pipeline_graph: histogram buffers are NULL");
    if (p->n_chunks_all == 0 || !any_active(p)) return HEPK_OK;
    int dev = 0;
    HEPK_HIP(hipGetDevice(&dev));
    HEPK_REQUIRE(dev == p->device, "hepk_pipeline_graph: plan made on device %d, current device %d", p->device, dev);
    const Launch L = make_launch(p, 0, p->n_chunks_all, sumw, counts);
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void *>(L.fn);
    kp.gridDim = dim3(L.grid);
    kp.blockDim = dim3(L.block);
    kp.sharedMemBytes = static_cast<unsigned int>(L.lds);
    PipeArgs a = L.a;
    void *kargs[] = {&a};
    kp.kernelParams = kargs;
    if (!p->gexec || p->gfn != L.fn || p->ggrid != L.grid) {
        if (p->gexec) HEPK_HIP(hipGraphExecDestroy(p->gexec));
        if (p->graph) HEPK_HIP(hipGraphDestroy(p->graph));
        p->gexec = nullptr;
        p->graph = nullptr;
        HEPK_HIP(hipGraphCreate(&p->graph, 0));
        HEPK_HIP(hipGraphAddKernelNode(&p->gnode, p->graph, nullptr, 0, &kp));
        HEPK_HIP(hipGraphInstantiate(&p->gexec, p->graph, nullptr, nullptr, 0));
    } else if (std::memcmp(&p->gargs, &a, sizeof(a)) != 0 || p->glds != L.lds) {
        HEPK_HIP(hipGraphExecKernelNodeSetParams(p->gexec, p->gnode, &kp));
    }
    p->gfn = L.fn;
    p->ggrid = L.grid;
    p->gargs = a;
    p->glds = L.lds;
    HEPK_HIP(hipGraphLaunch(p->gexec, stream));
    return HEPK_OK;
}

extern "C" int hepk_plan_destroy(hepk_plan p) {
    hepk::clear_error();
    if (!p) return HEPK_OK;
    if (!p->ring_ev.empty())
        for (size_t r = 0; r < p->ring_ev.size(); ++r)
            if (p->ring_used[r]) (void)hipEventSynchronize(p->ring_ev[r]);
    hepk::free_plan(p);
    return HEPK_OK;
}

extern "C" int hepk_autotune(const hepk_dataset *ds, int32_t n_ds, const hepk_query *q, int32_t n_query,
                             double *sumw, uint64_t *counts, int32_t reps, hepk_tune *best, float *best_ms,
                             hipStream_t stream) {
    using namespace hepk;
    clear_error();
    HEPK_REQUIRE(best && sumw && counts, "hepk_autotune: NULL argument");
    HEPK_REQUIRE(reps >= 1 && reps <= 1000, "hepk_autotune: reps %d out of [1, 1000]", reps);
    const hepk_tune cands[] = {{256, 1, 0, 0}, {512, 1, 0, 0}, {256, 2, 0, 0}, {512, 2, 0, 0},
                               {256, 1, 1, 0}, {512, 1, 1, 0}, {256, 2, 1, 0}, {512, 2, 1, 0}};
    hipEvent_t e0, e1;
    HEPK_HIP(hipEventCreate(&e0));
    HEPK_HIP(hipEventCreate(&e1));
    float best_t = INFINITY;
    hepk_tune best_c{};
    std::vector<hepk_tune> seen;
    int rc = HEPK_OK;
    for (const hepk_tune &c : cands) {
        hepk_plan p = nullptr;
        rc = hepk_plan_create(ds, n_ds, q, n_query, &c, &p);
        if (rc) break;
        hepk_tune eff{};
        hepk_plan_get_tune(p, &eff);
        bool dup = false;
        for (const auto &s : seen)
            dup |= s.block == eff.block && s.ev_per_thread == eff.ev_per_thread && s.hist_mode == eff.hist_mode;
        if (dup) {
            hepk_plan_destroy(p);
            continue;
        }
        seen.push_back(eff);
        std::vector<float> ts;
        rc = hepk_pipeline(p, sumw, counts, stream);  // warm-up
        for (int r = 0; rc == HEPK_OK && r < reps; ++r) {
            if (hipEventRecord(e0, stream) != hipSuccess) rc = HEPK_EHIP;
            if (rc == HEPK_OK) rc = hepk_pipeline(p, sumw, counts, stream);
            if (rc == HEPK_OK && hipEventRecord(e1, stream) != hipSuccess) rc = HEPK_EHIP;
            float ms = 0.0f;
            if (rc == HEPK_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = HEPK_EHIP;
            ts.push_back(ms);
        }
        hepk_plan_destroy(p);
        if (rc) break;
        std::sort(ts.begin(), ts.end());
        const float med = ts[ts.size() / 2];
        if (med < best_t) {
            best_t = med;
            best_c = eff;
            best_c.grid = 0;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    *best = best_c;
    if (best_ms) *best_ms = best_t;
    return HEPK_OK;
}
