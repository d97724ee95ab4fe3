// The fused analysis kernel of hepk_pipeline and its launch-shape table,
// shared by the translation units that instantiate it.
//
// The whole analysis pass of Sec. IV (object selection,
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
// with atomics).  A launch covers whole datasets (one chunk each); every
// workgroup takes an equal slice of their concatenated tiles, so uneven
// datasets never unbalance the launch, and merges its LDS histograms into
// HBM when its slice leaves a dataset.  For one tile a wavefront
//   1. reads the tile's object ranges with scalar loads (one tile ahead),
//      then issues all of its loads at once -- offsets (their low 32-bit
//      words) and weight of its events, up to JK jets, MK muons and EK
//      electrons per lane (consecutive lanes, consecutive objects:
//      coalesced) -- into registers, and waits once;
//   2. per query: muon (and electron) lanes evaluate the cuts; the selected
//      leptons are compacted by wavefront ballot into LDS in tile order,
//      with the count of selected leptons before each lepton;
//   3. each event lane writes its event's range of selected leptons over its
//      jets (an empty range for an event that cannot pass: too few selected
//      muons, or too few jets before any cut);
//   4. jet lanes test the cone against those leptons and store pt in LDS, or
//      NaN when removed, outside |eta|, or below jet_pt at every scale (the
//      last two skip the test);
//   5. event lanes walk their jets in order: ptv = pt * s, the jet cut, the
//      count, the left-to-right float32 H_T, the maximum, the b-tag count;
//      then the event cut and three fills into the workgroup's LDS
//      histograms (float64 sums, uint32 counts).  With several jet-energy
//      scales a lane takes an (event, group of kG scales) pair instead and
//      one walk serves the group.  The bins of all of a lane's fills are
//      found together (guesses, then every edge read, then the check).
// Steps 2-5 exchange data through the wavefront's own LDS region; a
// wavefront's LDS operations complete in issue order, so only compiler
// ordering fences are needed between them.  A tile whose objects exceed the
// register capacity (a 5-sigma fluctuation for the paper's multiplicities,
// always possible for arbitrary input) is processed one lane per event
// straight from HBM with the same arithmetic.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>

#include "common.hpp"
#include "lookup.hpp"

namespace hepk {

struct DsDev {
    int64_t n_events;
    const int64_t *joff, *moff, *eoff;
    const void *jpt, *jeta, *jphi, *jbt;
    const void *mpt, *meta, *mphi, *miso;
    const void *ept, *eeta, *ephi;
    const float *w;
    const float *npu;  // pileup per event (lookup weights); NULL: absent
    int64_t hist0;  // first slot of this dataset's block of histograms
    int64_t ev0;    // events of the datasets before this one (per-event records)
};

struct QDev {
    float mu_pt, mu_abseta, mu_iso, el_pt, el_abseta, jet_pt, jet_abseta, thr2, btag;
    int32_t min_mu, min_jet, min_b;
    int32_t n_scale, scale0;
    float smax;          // largest scale; used only when jet_pt >= 0
    int32_t active;      // 0: idle query slot, skipped
    int32_t nbins[3];
    int32_t ebase[3];    // first edge of each observable in the plan's edge table
    float lo[3], hi[3];  // first and last edge of each observable
    float inv_w[3];      // nbins / (hi - lo): start value of the bin search
    // The guess g = (x - lo) * inv_w (float32) can name a wrong bin only
    // where its fraction f = g - floor(g) has |f - 0.5| >= chk (a bound the
    // plan derives from the edges, guess_bounds); only such guesses are
    // checked against the edges.
    float chk[3];
    // Histogram of (scale v, observable h) starts at slot0 + v * per_scale +
    // hoff[h]: in the workgroup's LDS copy (compact over the active queries)
    // and in the dataset's block in HBM (fixed per query slot).
    int32_t lslot0, lper_scale, lhoff[3];
    int32_t gslot0, gper_scale, ghoff[3];
    // Lookup corrections (read by the LK kernels only).  Tables live in the
    // plan's edge table: pileup and muon scale-factor histograms (bins, first
    // edge, first slot content; pu_nb / sf_nb 0: that weight factor is
    // absent) and, with jes_mode 1, the jet-energy-scale shift table (rows of
    // |eta| bins, columns of pt bins, values row-major from jd); scales are
    // then shifts s with ptv = pt * (1 + s * delta).  smin: smallest scale.
    int32_t pu_nb, pu_e, pu_c, sf_nb, sf_e, sf_c;
    int32_t jes_mode, jr_nb, jr_e, jc_nb, jc_e, jd;
    float pu_lo, pu_hi, pu_iw, sf_lo, sf_hi, sf_iw;
    float jr_lo, jr_hi, jr_iw, jc_lo, jc_hi, jc_iw;
    float smin;
};

struct Chunk {
    int32_t d, pad;
    int64_t t0, t1;  // tiles [t0, t1) of dataset d
    int64_t pre;     // tiles of the chunks before this one
};

struct PipeArgs {
    const DsDev *ds;
    const QDev *qs;
    const float *scales;
    const Chunk *chunks;
    const float *edges;  // all queries' bin edges, concatenated
    int32_t chunk_begin, chunk_end;  // chunks [chunk_begin, chunk_end) of `chunks`
    int32_t n_q, ds_slots, n_edges, edges_in_lds;  // ds_slots: LDS histogram slots
    int32_t n_scales, scales_in_lds;               // the scale table, copied to LDS when small
    double *sumw;
    uint64_t *counts;
    double *sumw2;  // LK kernels: sums of squared weights (NULL: not kept)
    // per-event records (kernels instantiated with DBG only): the record of
    // event e of dataset d for scale v of query q is
    // rec[(q.scale0 + v) * rec_events + d.ev0 + e]
    hepk_event_record *rec;
    int64_t rec_events;
};

// Writes the record of one event and scale (DBG kernels only).
__device__ __forceinline__ hepk_event_record *rec_at(const PipeArgs &P, int row, int64_t ev) {
    return P.rec + static_cast<int64_t>(row) * P.rec_events + ev;
}

template <bool LDSH, bool W2 = false>
struct HistSink {
    double *sw;        // LDS (LDSH) or the dataset's block in HBM
    uint32_t *c32;     // LDS (LDSH)
    uint64_t *c64;     // HBM (!LDSH)
    double *sw2;       // W2: squared weights (LDS or HBM like sw; NULL: not kept)

    __device__ __forceinline__ void add(int slot, double w) const {
        atomic_add_f64(&sw[slot], w);
        if (W2 && sw2) atomic_add_f64(&sw2[slot], w * w);
        if (LDSH)
            atomicAdd(&c32[slot], 1u);
        else
            atomic_add_u64(&c64[slot], 1u);
    }
    // LDS histograms: adds w (and one count) where f holds and +0 / 0 where
    // it does not, without a branch (adding +0 changes no sum of finite
    // weights but a -0 one, which compares equal)
    __device__ __forceinline__ void add_if(int slot, double w, bool f) const {
        atomic_add_f64(&sw[slot], f ? w : 0.0);
        if (W2 && sw2) atomic_add_f64(&sw2[slot], f ? w * w : 0.0);
        atomicAdd(&c32[slot], f ? 1u : 0u);
    }
};

// The lookup tables of one query as axes over the edge table E.
struct LkAxes {
    Axis pu, sf, jr, jc;
};

template <typename QT>
__device__ __forceinline__ LkAxes lk_axes(const QT &Q, const float *E) {
    LkAxes a;
    a.pu = Axis{E + Q.pu_e, Q.pu_nb, Q.pu_lo, Q.pu_hi, Q.pu_iw};
    a.sf = Axis{E + Q.sf_e, Q.sf_nb, Q.sf_lo, Q.sf_hi, Q.sf_iw};
    a.jr = Axis{E + Q.jr_e, Q.jr_nb, Q.jr_lo, Q.jr_hi, Q.jr_iw};
    a.jc = Axis{E + Q.jc_e, Q.jc_nb, Q.jc_lo, Q.jc_hi, Q.jc_iw};
    return a;
}

// The jet-energy-scale shift of a jet (pt, eta) from the query's table.
__device__ __forceinline__ float jes_shift(const LkAxes &a, const float *E, int jd, float pt, float eta) {
    const int row = lookup_row(a.jr, fabsf(eta));
    return lookup_interp(a.jc, E + jd + (row - 1) * a.jc.nb, pt);
}

// jes_shift of N jets at once (lookup2_n over the query's table).
template <int N>
__device__ __forceinline__ void jes_shift_n(const LkAxes &a, const float *E, int jd, const float (&pt)[N],
                                            const float (&eta)[N], float (&out)[N]) {
    lookup2_n<N>(a.jr, a.jc, E + jd, pt, eta, out);
}

// Largest pt * (1 + s * d) over the scales in [smin, smax]: the factor is
// monotone in s (its rounding is monotone) and the product monotone in the
// factor, so the extremes are at smin or smax.  NaN when pt or d is NaN.
__device__ __forceinline__ float shifted_pt_bound(float pt, float d, float smin, float smax) {
    const float f_hi = 1.0f + smax * d, f_lo = 1.0f + smin * d;
    const float a = pt * f_hi, b = pt * f_lo;
    return (a != a) ? b : (b != b ? a : fmaxf(a, b));
}

// Histogram constants of one query, read once per query and held in
// registers: they are uniform, and without the pin the compiler reloads each
// field from memory (and waits for it) next to every use.
struct FillC {
    int32_t base, per;       // first slot of scale 0, slots per scale (LDS or global layout)
    int32_t nb[3], eb[3], off[3];
    float lo[3], hi[3], iw[3], ck[3];
};

template <typename X>
__device__ __forceinline__ X pin(X x) {
    asm volatile("" : "+s"(x));
    return x;
}

// All fields are read first and pinned by one statement, so their loads are
// issued together and waited for once (the guess bounds only with CERT).
template <bool LDSH, bool CERT, typename QT>
__device__ __forceinline__ FillC fill_consts(const QT &Q) {
    FillC F;
    F.base = LDSH ? Q.lslot0 : Q.gslot0;
    F.per = LDSH ? Q.lper_scale : Q.gper_scale;
#pragma unroll
    for (int h = 0; h < 3; ++h) {
        F.nb[h] = Q.nbins[h];
        F.eb[h] = Q.ebase[h];
        F.off[h] = LDSH ? Q.lhoff[h] : Q.ghoff[h];
        F.lo[h] = Q.lo[h];
        F.hi[h] = Q.hi[h];
        F.iw[h] = Q.inv_w[h];
        F.ck[h] = CERT ? Q.chk[h] : 0.0f;
    }
    asm volatile(""
                 : "+s"(F.base), "+s"(F.per), "+s"(F.nb[0]), "+s"(F.nb[1]), "+s"(F.nb[2]), "+s"(F.eb[0]),
                   "+s"(F.eb[1]), "+s"(F.eb[2]), "+s"(F.off[0]), "+s"(F.off[1]), "+s"(F.off[2]), "+s"(F.lo[0]),
                   "+s"(F.lo[1]), "+s"(F.lo[2]), "+s"(F.hi[0]), "+s"(F.hi[1]), "+s"(F.hi[2]), "+s"(F.iw[0]),
                   "+s"(F.iw[1]), "+s"(F.iw[2]));
    if (CERT) asm volatile("" : "+s"(F.ck[0]), "+s"(F.ck[1]), "+s"(F.ck[2]));
    return F;
}

// Slots of N values, x[n] going to observable n % 3 (H_T, lead, nJet): the
// same slot as hist_slot_lohi.  Without CERT every guess from the
// uniform-bin formula is checked against its bin's edges (one LDS round trip
// for all N values).  With CERT the guess is taken as exact unless its
// fraction is within the plan's bound of 0 or 1 (chk), so only lanes with such
// a guess read edges -- rarely any lane of a wavefront, so the round trip is
// usually skipped; this pays where a lane fills many values (several scales).
// Either way a binary search replaces a guess that was off.
template <int N, bool CERT>
__device__ __forceinline__ void find_bins(const FillC &F, const float *edges, const float (&x)[N], int (&s)[N]) {
    if (!CERT) {
        int k[N];
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const int h = n % 3;
            const float g = (x[n] - F.lo[h]) * F.iw[h];
            const int gi = g >= 0.0f ? (g < static_cast<float>(F.nb[h]) ? static_cast<int>(g) + 1 : F.nb[h]) : 1;
            s[n] = !(x[n] >= F.lo[h]) ? 0 : (x[n] >= F.hi[h] ? F.nb[h] + 1 : gi);
            k[n] = F.eb[h] + ((s[n] >= 1 && s[n] <= F.nb[h]) ? s[n] : 1);
        }
        float a[N], b[N];
#pragma unroll
        for (int n = 0; n < N; ++n) {
            a[n] = edges[k[n] - 1];
            b[n] = edges[k[n]];
        }
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const int h = n % 3;
            if (s[n] >= 1 && s[n] <= F.nb[h] && (x[n] < a[n] || x[n] >= b[n]))
                s[n] = bin_search(edges + F.eb[h], F.nb[h], x[n]);
        }
        return;
    }
    bool chk = false;  // some value of this lane needs the edges
#pragma unroll
    for (int n = 0; n < N; ++n) {
        // branch-free: the guess clamped to [0, nb - 1] before the
        // conversion (a NaN x clamps to 0 and lands in slot 0 below), the
        // predicates combined bitwise
        const int h = n % 3;
        const float g = (x[n] - F.lo[h]) * F.iw[h];
        const int gi = static_cast<int>(fminf(fmaxf(g, 0.0f), static_cast<float>(F.nb[h] - 1)));
        const int sv = x[n] >= F.hi[h] ? F.nb[h] + 1 : gi + 1;
        s[n] = x[n] >= F.lo[h] ? sv : 0;
        const float f = g - static_cast<float>(gi);
        chk |= (s[n] >= 1) & (s[n] <= F.nb[h]) &
               (!(g < static_cast<float>(F.nb[h])) | !(g >= 0.0f) | (fabsf(f - 0.5f) >= F.ck[h]));
    }
    if (chk) {
        // every value of the lane is verified (a right guess is kept)
#pragma unroll
        for (int n = 0; n < N; ++n) {
            const int h = n % 3;
            const float *E = edges + F.eb[h];
            if (s[n] >= 1 && s[n] <= F.nb[h] && (x[n] < E[s[n] - 1] || x[n] >= E[s[n]]))
                s[n] = bin_search(E, F.nb[h], x[n]);
        }
    }
}

// Fills H_T, lead and nJet of one passing event for scale v of query Q (a
// table entry read in place, so its fields are fetched where they are used).
template <bool LDSH, bool W2, typename QT>
__device__ __forceinline__ void fill3(const HistSink<LDSH, W2> &sink, const QT &Q, const float *edges, int v,
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

// One event, one lane, columns read straight from HBM.  LK: lookup event
// weights and, with jes_mode 1, shifted jet energies.
template <typename T, bool EXT, bool LDSH, bool DBG, bool LK>
__device__ void event_direct(const PipeArgs &P, const DsDev &D, int64_t e, const float *edges,
                             const HistSink<LDSH, LK> &sink) {
    const bool has_iso = D.miso != nullptr;
    const bool has_el = EXT && D.eoff != nullptr;
    const bool has_bt = EXT && D.jbt != nullptr;
    const float w0 = D.w ? D.w[e] : 1.0f;
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
        // event weight: w, times the pileup lookup, times the product (left
        // to right from 1) of the selected muons' scale factors
        float wq = w0;
        LkAxes ax{};
        if (LK) {
            ax = lk_axes(Q, edges);
            if (Q.pu_nb > 0 && D.npu) wq = wq * lookup_bin(ax.pu, edges + Q.pu_c, D.npu[e]);
            if (Q.sf_nb > 0) {
                float prod = 1.0f;
                for (int64_t m = m0; m < m1; ++m)
                    if (mu_sel(m)) prod = prod * lookup_bin(ax.sf, edges + Q.sf_c, ldf(mpt, m));
                wq = wq * prod;
            }
        }
        const bool shift = LK && Q.jes_mode == 1;
        for (int v = 0; v < Q.n_scale; ++v) {
            const float s = as_const(P.scales)[Q.scale0 + v];
            int nj = 0, nb = 0;
            float ht = 0.0f, lead = -INFINITY;
            for (int64_t j = j0; j < j1; ++j) {
                const float pt = ldf(jpt, j);
                const float eta = ldf(jeta, j);
                const float x = shift ? pt * (1.0f + s * jes_shift(ax, edges, Q.jd, pt, eta)) : pt * s;
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
            if (DBG)
                *rec_at(P, Q.scale0 + v, D.ev0 + e) = hepk_event_record{nmu, nj, nb, pass ? 3 : 2, ht, lead, wq, 0};
            if (pass) fill3(sink, Q, edges, v, ht, lead, nj, static_cast<double>(wq));
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
    // both lepton ranges of a jet in one word (8-bit first and count each)
    // when the tile caps allow it
    static constexpr bool PACK = EXT && MC <= 255 && EC <= 255;
};

// One wavefront's LDS.  jr holds, per jet, its event's range of selected
// muons (first | count << 16; with PACK, muons in the low and electrons in
// the high 16 bits, first | count << 8 each) until the cone test reads it;
// the same word then holds the jet's pt (or NaN) for the per-event walk
// (with one scale and jet_pt >= 0: pt * s of a selected jet, else +0).
// The selected muons and (extended schema) electrons share one pair of
// arrays, the electrons from index EO = MC + 2 on, so one index runs over an
// event's muons and then its electrons.
// With several scales (MS) the cone test instead compacts the jets that can
// be selected at some scale (the candidates) into jr, bt and jd in tile
// order, and cpre[j] holds the number of candidates (low 16 bits) and of
// b-tagged candidates (high 16 bits) before tile jet j; cpre shares space
// with the compacted leptons, which are dead by then.
template <int EVPL, bool EXT, bool LK, bool MS>
struct WaveLds {
    using C = Caps<EVPL, EXT>;
    union {
        uint32_t rng;
        float pt;
    } jr[C::JC];
    uint32_t jre[(EXT && !C::PACK) ? C::JC : 1];  // electron ranges when not packed
    union {
        struct {
            // selected muons, compacted in tile order (+2 padding), then
            // (EXT) the selected electrons likewise from index EO
            float seta[C::MC + 2 + (EXT ? C::EC + 2 : 0)], sphi[C::MC + 2 + (EXT ? C::EC + 2 : 0)];
            float ssf[LK ? C::MC + 2 : 1];  // LK: selected muons' scale factors, compacted like seta
        };
        uint32_t cpre[MS ? C::JC + 1 : 1];
    };
    float jd[LK ? C::JC : 1];       // LK: each jet's energy-scale shift (jes_mode 1)
    uint8_t bt[EXT ? C::JC : 1];
    union {
        struct {  // steps 2-3: selected leptons before lepton m
            uint16_t mpre[C::MC + 1];
            uint16_t epre[EXT ? C::EC + 1 : 1];
        } p;
        struct {  // step 5, several scales: eligible events (compacted),
                  // jet range (first | end << 16) and weight
            uint32_t evjr[C::TW];
            float evw[C::TW];
        } w;
    } u;
};

// Adds weight w to the histograms of scales v0 + n / 3 (observable n % 3)
// of the lanes whose pass[n / 3] is set; NaN values are not filled.  With
// several scales and LDS histograms every lane adds, zero where it does not
// fill, at a slot of a scale no later than vlast (the query's last), so no
// value needs its own branch.
template <int N, bool CERT, bool LDSH, bool W2>
__device__ __forceinline__ void fill_bins(const HistSink<LDSH, W2> &sink, const FillC &F, const float *edges,
                                          const float (&xs)[N], const bool (&pass)[N / 3], int v0, double w,
                                          int vlast) {
    int sl[N];
    find_bins<N, CERT>(F, edges, xs, sl);
    if (CERT && LDSH) {
#pragma unroll
        for (int n = 0; n < N; ++n)
            sink.add_if(F.base + min(v0 + n / 3, vlast) * F.per + F.off[n % 3] + sl[n], w,
                        pass[n / 3] & (xs[n] == xs[n]));
        return;
    }
#pragma unroll
    for (int n = 0; n < N; ++n)
        if (pass[n / 3] && xs[n] == xs[n]) sink.add(F.base + (v0 + n / 3) * F.per + F.off[n % 3] + sl[n], w);
}

// Scales per lane in the walk over an event's jets when a query has several
// (even: the fills take them two at a time).
constexpr int kG = 4;

// Walks the jets [j0, j1) of one event in order (pt of each in LDS, NaN when
// removed by the cone or |eta| cut) for G scales at once: per scale the
// left-to-right float32 H_T of the selected jets (ptv > jet_pt), their
// count, b-tag count and maximum.  Adding only selected values keeps the sum
// order of the definition.  ptv = pt * s, or with JM (shifted energies)
// pt * (1 + s * d) with the jet's shift d from LDS.  For ptv = pt * s the
// maximum needs no per-scale work: for s > 0, rounding pt * s is monotone
// in pt, so the selected jets are those above a pt bound and the largest
// selected pt * s is the largest cleaned pt times s (rounded once), whenever
// any jet is selected; with JM the factor differs per jet and the maximum is
// taken per scale.  Branch-free, two jets per step (both LDS reads in
// flight).
template <int G, bool EXT, bool JM, typename WL>
__device__ __forceinline__ void walk_jets(const WL &L, int j0, int j1, const float (&sc)[G], float jet_pt,
                                          float (&ht)[G], float (&lead)[G], int (&nj)[G], int (&nb)[G]) {
    float pmax = -INFINITY;
    // selected jets (low 16 bits) and selected b-tagged jets (high 16 bits)
    // in one counter per scale: a range holds at most 64 * JK < 2^16 jets
    uint32_t cnt[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        ht[g] = 0.0f;
        cnt[g] = 0u;
        lead[g] = -INFINITY;
    }
    auto step = [&](float p, float d, int bt) {
        pmax = fmaxf(pmax, p);  // NaN (removed jet) leaves it unchanged
        const uint32_t inc = EXT ? 1u + (static_cast<uint32_t>(bt) << 16) : 1u;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const float f = JM ? 1.0f + sc[g] * d : sc[g];
            const float x = p * f;
            const bool sel = x > jet_pt;
            const float hs = ht[g] + x;
            ht[g] = sel ? hs : ht[g];
            cnt[g] += sel ? inc : 0u;
            if (JM) lead[g] = sel ? fmaxf(lead[g], x) : lead[g];
        }
    };
    int k = j0;
    for (; k + 2 <= j1; k += 2) {
        const float p0 = L.jr[k].pt, p1 = L.jr[k + 1].pt;
        const float d0 = JM ? L.jd[k] : 0.0f, d1 = JM ? L.jd[k + 1] : 0.0f;
        const int b0 = EXT ? L.bt[k] : 0, b1 = EXT ? L.bt[k + 1] : 0;
        step(p0, d0, b0);
        step(p1, d1, b1);
    }
    if (k < j1) step(L.jr[k].pt, JM ? L.jd[k] : 0.0f, EXT ? static_cast<int>(L.bt[k]) : 0);
#pragma unroll
    for (int g = 0; g < G; ++g) {
        nj[g] = static_cast<int>(cnt[g] & 0xffffu);
        nb[g] = EXT ? static_cast<int>(cnt[g] >> 16) : 0;
        if (!JM) lead[g] = nj[g] > 0 ? pmax * sc[g] : -INFINITY;
    }
}

// The same reductions for one scale s when the cone test already stored
// every selected jet as pt * s and every other jet as +0 (possible when
// jet_pt >= 0: a selected value exceeds jet_pt >= 0, so it is positive and
// the count is that of positive values).  Adding +0 leaves a float32 sum of
// positive values unchanged, so summing every stored value keeps the sum
// order of the definition.  The b-tag flag is stored already ANDed with the
// selection.
template <bool EXT, typename WL>
__device__ __forceinline__ void walk_selected(const WL &L, int j0, int j1, float &ht, float &lead, int &nj,
                                              int &nb) {
    float h = 0.0f, m = 0.0f;
    int n = 0, b = 0;
    auto step = [&](float x, int bt) {
        h += x;
        n += x > 0.0f ? 1 : 0;
        m = fmaxf(m, x);
        if (EXT) b += bt;
    };
    int k = j0;
    for (; k + 2 <= j1; k += 2) {
        const float x0 = L.jr[k].pt, x1 = L.jr[k + 1].pt;
        const int b0 = EXT ? L.bt[k] : 0, b1 = EXT ? L.bt[k + 1] : 0;
        step(x0, b0);
        step(x1, b1);
    }
    if (k < j1) step(L.jr[k].pt, EXT ? static_cast<int>(L.bt[k]) : 0);
    ht = h;
    nj = n;
    nb = b;
    lead = n > 0 ? m : -INFINITY;
}

// A tile's first object of each collection and its object counts (32-bit:
// the counts are what the kernel compares and indexes with).
struct TileBounds {
    int64_t J0, M0, L0;
    int32_t nj, nm, nl;
};

template <bool EXT, typename DT>
__device__ __forceinline__ TileBounds tile_bounds(const DT &D, bool has_el, int64_t e0, int ne) {
    TileBounds b;
    b.J0 = as_const(D.joff)[e0];
    b.nj = static_cast<int32_t>(as_const(D.joff)[e0 + ne] - b.J0);
    b.M0 = as_const(D.moff)[e0];
    b.nm = static_cast<int32_t>(as_const(D.moff)[e0 + ne] - b.M0);
    b.L0 = (EXT && has_el) ? as_const(D.eoff)[e0] : 0;
    b.nl = (EXT && has_el) ? static_cast<int32_t>(as_const(D.eoff)[e0 + ne] - b.L0) : 0;
    return b;
}

// Compacts the selected objects of a tile (sel per slot k of this lane) into
// (eta, phi) arrays in tile order (and, with V3, a third value into o3);
// pre[m] = number of selected objects before object m, pre[n] = total.
template <int K, bool V3 = false>
__device__ __forceinline__ void compact(const bool (&sel)[K], const float (&eta)[K], const float (&phi)[K], int n,
                                        int lane, float *oeta, float *ophi, uint16_t *pre,
                                        const float *v3 = nullptr, float *o3 = nullptr) {
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
            if (V3) o3[before] = v3[k];
        }
        run += __popcll(bal);
    }
    if (lane == 0) pre[n] = static_cast<uint16_t>(run);
}

// MS: the plan has queries with several jet-energy scales (every query then
// takes the scale-group walk of step 5; otherwise every query has one scale).
// Occupancy targets: base schema, one scale: six wavefronts per SIMD (at most
// 80 VGPRs), measured the best trade between latency hiding and the
// registers that hold a tile in flight; extended schema: four (its
// wavefronts need twice the LDS); several scales: two, which is what LDS
// allows next to the histograms of 20 scales, so the walk and the fills
// may use the registers for instruction-level parallelism instead.
// DBG: also write every event's per-scale record (counts, H_T, leading pt,
// whether the event was walked and whether it passed) to P.rec -- the
// intermediate values of the pass, for checking them one by one.  Product
// launches use DBG = false; the arithmetic is the same in both.
// LK: the lookup corrections of Sec. IV -- event weights from the pileup and
// muon scale-factor lookup histograms, jet energies shifted by an
// interpolated table (jes_mode 1) -- and the sums of squared weights; a
// query without lookups runs exactly as in the kernels without LK.
template <typename T, bool EXT, int WAVES, int EVPL, bool LDSH, bool MS, bool DBG, bool LK>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(MS ? 2 : (EXT || LK ? 4 : 6)))) void
pipeline_kernel(PipeArgs P) {
    using C = Caps<EVPL, EXT>;
    constexpr int TW = C::TW, JK = C::JK, MK = C::MK, EK = C::EK;
    __shared__ WaveLds<EVPL, EXT, LK, MS> wl[WAVES];
    // per workgroup: [sumw | sumw2 (LK) | counts (u32) | edges | scales]
    extern __shared__ double dyn[];

    const int tid = threadIdx.x;
    int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    auto &L = wl[wave];

    double *sw_s = dyn;
    double *sw2_s = dyn + (LDSH ? P.ds_slots : 0);
    uint32_t *c_s = reinterpret_cast<uint32_t *>(sw2_s + ((LDSH && LK) ? P.ds_slots : 0));
    float *e_s = reinterpret_cast<float *>(c_s + (LDSH ? P.ds_slots : 0));
    if (LDSH) {
        for (int i = tid; i < P.ds_slots; i += 64 * WAVES) {
            sw_s[i] = 0.0;
            if (LK) sw2_s[i] = 0.0;
            c_s[i] = 0u;
        }
    }
    float *s_s = e_s + (P.edges_in_lds ? P.n_edges : 0);
    const float *edges = P.edges;
    if (P.edges_in_lds) {
        for (int i = tid; i < P.n_edges; i += 64 * WAVES) e_s[i] = as_const(P.edges)[i];
        edges = e_s;
    }
    if (P.scales_in_lds)
        for (int i = tid; i < P.n_scales; i += 64 * WAVES) s_s[i] = as_const(P.scales)[i];
    __syncthreads();
    // Runs f on the table (edges and lookup tables) where it lives, with a
    // pointer whose address space the compiler can see (LDS reads rather
    // than flat ones).
    auto on_tables = [&](auto &&f) {
        if (P.edges_in_lds)
            f(static_cast<const float *>(e_s));
        else
            f(static_cast<const float *>(P.edges));
    };

    // This workgroup's work: an equal slice [my0, my1) of the concatenated
    // tiles of chunks [chunk_begin, chunk_end); its first chunk is found by a
    // binary search over the chunks' tile prefixes (uniform, scalar loads).
    const auto chs = as_const(P.chunks);
    const int64_t T0 = chs[P.chunk_begin].pre;
    const int64_t nT = chs[P.chunk_end - 1].pre + (chs[P.chunk_end - 1].t1 - chs[P.chunk_end - 1].t0) - T0;
    const int64_t my0 = T0 + nT * blockIdx.x / gridDim.x;
    const int64_t my1 = T0 + nT * (blockIdx.x + 1) / gridDim.x;
    int qlast = -1;  // the last active query (its cone test ends a tile's use of the columns)
    for (int q = 0; q < P.n_q; ++q)
        if (as_const(P.qs)[q].active) qlast = q;
    int cfirst = P.chunk_begin;
    for (int hi = P.chunk_end - 1; cfirst < hi;) {  // last chunk with pre <= my0
        const int mid = (cfirst + hi + 1) >> 1;
        if (chs[mid].pre <= my0)
            cfirst = mid;
        else
            hi = mid - 1;
    }
    for (int ci = cfirst; ci < P.chunk_end && my0 < my1; ++ci) {
        const Chunk CH = chs[ci];
        if (CH.pre >= my1) break;
        // this workgroup's tiles of the chunk
        const int64_t c_t0 = CH.t0 + max<int64_t>(my0 - CH.pre, 0);
        const int64_t c_t1 = CH.t0 + min<int64_t>(my1 - CH.pre, CH.t1 - CH.t0);
        if (c_t1 <= c_t0) continue;
        const auto &D = as_const(P.ds)[CH.d];  // read in place, like the query table
        HistSink<LDSH, LK> sink;
        if (LDSH) {
            sink.sw = sw_s;
            sink.c32 = c_s;
            sink.sw2 = (LK && P.sumw2) ? sw2_s : nullptr;
        } else {
            sink.sw = P.sumw + D.hist0;
            sink.c64 = P.counts + D.hist0;
            sink.sw2 = (LK && P.sumw2) ? P.sumw2 + D.hist0 : nullptr;
        }
        const bool has_iso = D.miso != nullptr;
        const bool has_el = EXT && D.eoff != nullptr;
        const bool has_bt = EXT && D.jbt != nullptr;

        // several scales: the next (sub-)tile's loads fly during the walks and
        // fills (see the tile loop below) -- where the registers allow it
        // (LDS histograms, workgroups of at most 512 threads, one event per
        // lane: up to 256 VGPRs; the other shapes would spill)
        constexpr bool PIPE = MS && LDSH && WAVES <= 8 && EVPL == 1;
        // The raw loads of one tile (the offsets as their low 32-bit words:
        // tile-relative differences are exact modulo 2^32).
        // (content as raw bits: float32, or float16 in the low half)
        struct Raw {
            uint32_t j0[EVPL], j1[EVPL], m0[EVPL], m1[EVPL], l0[EVPL], l1[EVPL];
            float w[EVPL];
            float npu[LK ? EVPL : 1];
            uint32_t jpt[JK], jeta[JK], jphi[JK], jbt[EXT ? JK : 1];
            uint32_t mpt[MK], meta[MK], mphi[MK], miso[MK];
            uint32_t lpt[EK], leta[EK], lphi[EK];
        };
        // The chunk's tiles are counted from c_t0 in 32 bits (a workgroup's
        // share of one dataset has far fewer than 2^31 tiles); only the last
        // one can hold fewer than TW events.
        const int nt = static_cast<int>(c_t1 - c_t0);
        const int64_t ebase = c_t0 * TW;
        const int tn_last = static_cast<int>(min<int64_t>(TW, D.n_events - (c_t1 - 1) * TW));
        auto tile_events = [&](int r) { return r == nt - 1 ? tn_last : TW; };
        auto bounds_of = [&](int r) {
            return tile_bounds<EXT>(D, has_el, ebase + static_cast<int64_t>(r) * TW, tile_events(r));
        };
        // (compared unsigned: a count of 2^31 to 2^32 objects, which valid
        // offsets of one tile never give, also goes the per-event way)
        auto oversize = [&](const TileBounds &b) {
            return static_cast<uint32_t>(b.nj) > static_cast<uint32_t>(C::JC) ||
                   static_cast<uint32_t>(b.nm) > static_cast<uint32_t>(C::MC) ||
                   static_cast<uint32_t>(b.nl) > static_cast<uint32_t>(C::EC);
        };
        // ---- 1. all of a tile's loads, without waiting: both offsets of each
        // event lane's event (their low 32-bit words), its weight, and up to
        // JK jets, MK muons and EK electrons per lane (consecutive lanes,
        // consecutive objects).  Buffer loads over exactly the tile's range
        // of each column read 0 past its end, which is the value every
        // unused slot must hold.
        auto issue = [&](int64_t e0, int ne, const TileBounds &b, Raw &R) {
            // the extended schema measured 1.5% faster with nontemporal loads,
            // the base schema 1.3% slower
            constexpr int AUX = EXT ? kBufNt : 0;
            const int nj = b.nj, nm = b.nm, nl = b.nl;
            // offsets: events e0 .. e0 + ne (both ends of each event)
            const uint32_t ob = static_cast<uint32_t>(ne + 1) * 8u;
            const buf_t bjo = buf_span(D.joff + e0, ob), bmo = buf_span(D.moff + e0, ob);
            const buf_t beo = buf_span((EXT && has_el) ? D.eoff + e0 : D.joff + e0, ob);
            const buf_t bw = buf_span(D.w ? static_cast<const void *>(D.w + e0) : D.joff, static_cast<uint32_t>(ne) * 4u);
            const buf_t bpu =
                buf_span(LK && D.npu ? static_cast<const void *>(D.npu + e0) : D.joff, static_cast<uint32_t>(ne) * 4u);
#pragma unroll
            for (int r = 0; r < EVPL; ++r) {
                const int ev = lane + 64 * r;
                R.j0[r] = buf_u32<AUX>(bjo, ev * 8);
                R.j1[r] = buf_u32<AUX>(bjo, ev * 8 + 8);
                R.m0[r] = buf_u32<AUX>(bmo, ev * 8);
                R.m1[r] = buf_u32<AUX>(bmo, ev * 8 + 8);
                R.l0[r] = R.l1[r] = 0;
                if (EXT && has_el) {
                    R.l0[r] = buf_u32<AUX>(beo, ev * 8);
                    R.l1[r] = buf_u32<AUX>(beo, ev * 8 + 8);
                }
                R.w[r] = D.w ? __builtin_bit_cast(float, buf_u32<AUX>(bw, ev * 4)) : 1.0f;
                if (LK) R.npu[LK ? r : 0] = D.npu ? __builtin_bit_cast(float, buf_u32<AUX>(bpu, ev * 4)) : 0.0f;
            }
            const uint32_t es = sizeof(T);
            const buf_t bjpt = buf_span(static_cast<const T *>(D.jpt) + b.J0, nj * es);
            const buf_t bjeta = buf_span(static_cast<const T *>(D.jeta) + b.J0, nj * es);
            const buf_t bjphi = buf_span(static_cast<const T *>(D.jphi) + b.J0, nj * es);
#pragma unroll
            for (int k = 0; k < JK; ++k) {
                const int j = lane + 64 * k;
                R.jpt[k] = buf_raw<T, AUX>(bjpt, j);
                R.jeta[k] = buf_raw<T, AUX>(bjeta, j);
                R.jphi[k] = buf_raw<T, AUX>(bjphi, j);
                if (EXT) R.jbt[EXT ? k : 0] = 0u;
            }
            if (EXT && has_bt) {
                const buf_t bjbt = buf_span(static_cast<const T *>(D.jbt) + b.J0, nj * es);
#pragma unroll
                for (int k = 0; k < JK; ++k) R.jbt[EXT ? k : 0] = buf_raw<T, AUX>(bjbt, lane + 64 * k);
            }
            const buf_t bmpt = buf_span(static_cast<const T *>(D.mpt) + b.M0, nm * es);
            const buf_t bmeta = buf_span(static_cast<const T *>(D.meta) + b.M0, nm * es);
            const buf_t bmphi = buf_span(static_cast<const T *>(D.mphi) + b.M0, nm * es);
#pragma unroll
            for (int k = 0; k < MK; ++k) {
                const int m = lane + 64 * k;
                R.mpt[k] = buf_raw<T, AUX>(bmpt, m);
                R.meta[k] = buf_raw<T, AUX>(bmeta, m);
                R.mphi[k] = buf_raw<T, AUX>(bmphi, m);
                R.miso[k] = 0u;
            }
            if (has_iso) {
                const buf_t bmiso = buf_span(static_cast<const T *>(D.miso) + b.M0, nm * es);
#pragma unroll
                for (int k = 0; k < MK; ++k) R.miso[k] = buf_raw<T, AUX>(bmiso, lane + 64 * k);
            }
#pragma unroll
            for (int k = 0; k < EK; ++k) R.lpt[k] = R.leta[k] = R.lphi[k] = 0u;
            if (EXT && has_el) {
                const buf_t bept = buf_span(static_cast<const T *>(D.ept) + b.L0, nl * es);
                const buf_t beeta = buf_span(static_cast<const T *>(D.eeta) + b.L0, nl * es);
                const buf_t bephi = buf_span(static_cast<const T *>(D.ephi) + b.L0, nl * es);
#pragma unroll
                for (int k = 0; k < EK; ++k) {
                    const int m = lane + 64 * k;
                    R.lpt[k] = buf_raw<T, AUX>(bept, m);
                    R.leta[k] = buf_raw<T, AUX>(beeta, m);
                    R.lphi[k] = buf_raw<T, AUX>(bephi, m);
                }
            }
        };
        // Every value of R is used here, so the compiler waits for the tile's
        // loads at this point (once), not at each value's first use.
        auto settle = [&](Raw &R) {
#pragma unroll
            for (int r = 0; r < EVPL; ++r)
                asm volatile("" ::"v"(R.j0[r]), "v"(R.j1[r]), "v"(R.m0[r]), "v"(R.m1[r]), "v"(R.w[r]));
            if (LK) {
#pragma unroll
                for (int r = 0; r < EVPL; ++r) asm volatile("" ::"v"(R.npu[LK ? r : 0]));
            }
#pragma unroll
            for (int k = 0; k < JK; ++k) asm volatile("" ::"v"(R.jpt[k]), "v"(R.jeta[k]), "v"(R.jphi[k]));
#pragma unroll
            for (int k = 0; k < MK; ++k)
                asm volatile("" ::"v"(R.mpt[k]), "v"(R.meta[k]), "v"(R.mphi[k]), "v"(R.miso[k]));
            if (EXT) {
#pragma unroll
                for (int r = 0; r < EVPL; ++r) asm volatile("" ::"v"(R.l0[r]), "v"(R.l1[r]));
#pragma unroll
                for (int k = 0; k < JK; ++k) asm volatile("" ::"v"(R.jbt[EXT ? k : 0]));
#pragma unroll
                for (int k = 0; k < EK; ++k) asm volatile("" ::"v"(R.lpt[k]), "v"(R.leta[k]), "v"(R.lphi[k]));
            }
        };
        // Steps 2-5 for every query on a settled tile.
        auto work = [&](int64_t e0, int ne, const TileBounds &B, Raw &R, auto &&after_cone) {
            const int nj = B.nj, nm = B.nm, nl = B.nl;
            int32_t jb[EVPL], je[EVPL], mb[EVPL], me[EVPL], lb[EVPL], le[EVPL];
            float wv[EVPL];
#pragma unroll
            for (int r = 0; r < EVPL; ++r) {
                const bool in = lane + 64 * r < ne;
                jb[r] = in ? static_cast<int32_t>(R.j0[r] - static_cast<uint32_t>(B.J0)) : 0;
                je[r] = in ? static_cast<int32_t>(R.j1[r] - static_cast<uint32_t>(B.J0)) : 0;
                mb[r] = in ? static_cast<int32_t>(R.m0[r] - static_cast<uint32_t>(B.M0)) : 0;
                me[r] = in ? static_cast<int32_t>(R.m1[r] - static_cast<uint32_t>(B.M0)) : 0;
                lb[r] = (in && EXT && has_el) ? static_cast<int32_t>(R.l0[r] - static_cast<uint32_t>(B.L0)) : 0;
                le[r] = (in && EXT && has_el) ? static_cast<int32_t>(R.l1[r] - static_cast<uint32_t>(B.L0)) : 0;
                wv[r] = R.w[r];
            }
            float jpt[JK], jeta[JK], jphi[JK], jbt[EXT ? JK : 1];
            float mpt[MK], meta[MK], mphi[MK], miso[MK];
            float lpt[EK], leta[EK], lphi[EK];
#pragma unroll
            for (int k = 0; k < JK; ++k) {
                jpt[k] = raw_f<T>(R.jpt[k]);
                jeta[k] = raw_f<T>(R.jeta[k]);
                jphi[k] = raw_f<T>(R.jphi[k]);
                if (EXT) jbt[EXT ? k : 0] = raw_f<T>(R.jbt[EXT ? k : 0]);
            }
#pragma unroll
            for (int k = 0; k < MK; ++k) {
                mpt[k] = raw_f<T>(R.mpt[k]);
                meta[k] = raw_f<T>(R.meta[k]);
                mphi[k] = raw_f<T>(R.mphi[k]);
                miso[k] = raw_f<T>(R.miso[k]);
            }
#pragma unroll
            for (int k = 0; k < EK; ++k) {
                lpt[k] = raw_f<T>(R.lpt[k]);
                leta[k] = raw_f<T>(R.leta[k]);
                lphi[k] = raw_f<T>(R.lphi[k]);
            }
            (void)jbt;
            (void)lpt;
            for (int q = 0; q < P.n_q; ++q) {
                // (values derived from the lane index are recomputed per
                // query rather than held across the query loop)
                asm volatile("" : "+v"(lane));
                // the query's fields are read in place (scalar loads near their
                // uses) rather than copied: a copy would hold ~45 SGPRs for the
                // whole query and spill
                const auto &Q = as_const(P.qs)[q];
                if (!Q.active) continue;
                // the query's cut constants, read once and pinned by one
                // statement (loads issued together, one wait; unpinned, the
                // compiler reloads them inside the loops below, a wait each)
                float mu_pt = Q.mu_pt, mu_abseta = Q.mu_abseta, mu_iso = Q.mu_iso;
                float el_pt = EXT ? Q.el_pt : 0.0f, el_abseta = EXT ? Q.el_abseta : 0.0f;
                float jet_pt = Q.jet_pt, thr2 = Q.thr2, jet_abseta = Q.jet_abseta, smax = Q.smax;
                float btag = EXT ? Q.btag : 0.0f;
                int min_mu = Q.min_mu, min_jet = Q.min_jet, min_b = has_bt ? Q.min_b : 0;
                asm volatile(""
                             : "+s"(mu_pt), "+s"(mu_abseta), "+s"(mu_iso), "+s"(el_pt), "+s"(el_abseta),
                               "+s"(jet_pt), "+s"(thr2), "+s"(jet_abseta), "+s"(smax), "+s"(btag), "+s"(min_mu),
                               "+s"(min_jet), "+s"(min_b));
                // lookup corrections of this query (LK kernels): which are on,
                // the tables as axes over the edge table
                const bool use_pu = LK && Q.pu_nb > 0 && D.npu != nullptr;
                const bool use_sf = LK && Q.sf_nb > 0;
                const bool shift = LK && Q.jes_mode == 1;
                const float smin = LK ? Q.smin : 0.0f;
                // ---- 2. lepton selection; selected leptons compacted into LDS
                // (all compares evaluated: no branches per slot)
                {
                    bool sel[MK];
#pragma unroll
                    for (int k = 0; k < MK; ++k)
                        sel[k] = (lane + 64 * k < nm) & (mpt[k] > mu_pt) & (fabsf(meta[k]) < mu_abseta) &
                                 (!has_iso | (miso[k] < mu_iso));
                    if (use_sf) {
                        // each selected muon's scale factor, compacted beside it
                        float sfv[MK];
                        on_tables([&](const float *E) { lookup_bin_n<MK>(lk_axes(Q, E).sf, E + Q.sf_c, mpt, sel, sfv, false); });
                        compact<MK, true>(sel, meta, mphi, nm, lane, L.seta, L.sphi, L.u.p.mpre, sfv, L.ssf);
                    } else {
                        compact<MK>(sel, meta, mphi, nm, lane, L.seta, L.sphi, L.u.p.mpre);
                    }
                }
                if (EXT) {
                    bool sel[EK];
#pragma unroll
                    for (int k = 0; k < EK; ++k)
                        sel[k] = (lane + 64 * k < nl) & (lpt[k] > el_pt) & (fabsf(leta[k]) < el_abseta);
                    compact<EK>(sel, leta, lphi, nl, lane, L.seta + (C::MC + 2), L.sphi + (C::MC + 2), L.u.p.epre);
                }
                wave_sync();
                // ---- 3. each event lane writes its selected-lepton range over
                // its jets; an event that cannot pass (too few muons, or too
                // few jets before any cut) gets empty ranges: its jets' cone
                // test is not needed
                int nmu[EVPL];
                float wq[EVPL];  // the event weight of this query
#pragma unroll
                for (int r = 0; r < EVPL; ++r) {
                    nmu[r] = 0;
                    wq[r] = wv[r];
                    const int ev = lane + 64 * r;
                    if (ev < ne) {
                        const int s0 = L.u.p.mpre[mb[r]];
                        nmu[r] = L.u.p.mpre[me[r]] - s0;
                        if (use_pu)
                            on_tables([&](const float *E) {
                                wq[r] = wq[r] * lookup_bin(lk_axes(Q, E).pu, E + Q.pu_c, R.npu[LK ? r : 0]);
                            });
                        if (use_sf) {
                            // product of the selected muons' scale factors, in order from 1
                            float prod = 1.0f;
                            for (int i = s0; i < s0 + nmu[r]; ++i) prod = prod * L.ssf[i];
                            wq[r] = wq[r] * prod;
                        }
                        const bool elig = nmu[r] >= min_mu && je[r] - jb[r] >= min_jet;
                        constexpr int CS = C::PACK ? 8 : 16;  // count shift
                        uint32_t pk = static_cast<uint32_t>(s0) | (static_cast<uint32_t>(elig ? nmu[r] : 0) << CS);
                        uint32_t pke = 0;
                        if (EXT) {
                            const int u0 = L.u.p.epre[lb[r]];
                            pke = static_cast<uint32_t>(u0) |
                                  (static_cast<uint32_t>(elig ? L.u.p.epre[le[r]] - u0 : 0) << CS);
                            if (C::PACK) pk |= pke << 16;
                        }
                        // two jets per step (a divergent loop: its trip count
                        // is the largest jet count of the wavefront)
                        int k = jb[r];
                        for (; k + 2 <= je[r]; k += 2) {
                            L.jr[k].rng = pk;
                            L.jr[k + 1].rng = pk;
                            if (EXT && !C::PACK) {
                                L.jre[C::PACK ? 0 : k] = pke;
                                L.jre[C::PACK ? 0 : k + 1] = pke;
                            }
                        }
                        if (k < je[r]) {
                            L.jr[k].rng = pk;
                            if (EXT && !C::PACK) L.jre[C::PACK ? 0 : k] = pke;
                        }
                    }
                }
                wave_sync();
                // ---- 4. cone test per jet against its event's selected
                // leptons.  A jet outside |eta| or below jet_pt at the largest
                // scale (with jet_pt >= 0) is selected at no scale: it skips
                // the test and is stored as NaN.  That changes no result: a
                // selected jet of its event has a larger pt, so the maximum
                // and the sums and counts of selected jets are the same.
                // With one scale and jet_pt >= 0 (zsel) this step decides the
                // whole jet selection, so a kept jet is stored as pt * s and
                // any other as +0, for walk_selected.
                const bool zsel = !MS && jet_pt >= 0.0f;
                // Slots in pairs (CB; three at a time spills registers): the
                // pair's packed ranges, then the first two selected leptons of
                // each slot's event, each set of reads in flight together (two
                // LDS round trips per pair); only events with more leptons loop
                // over the rest.  An event's leptons are its selected muons,
                // then (EXT) its selected electrons: lepton i is seta[s0 + i]
                // for i < nmu, else seta[EO + u0 + i - nmu].  A slot past the
                // tile's jets reads a stale word: its firsts and counts are
                // forced to 0.  Reads past a range's end land on other
                // events' leptons or on the padding entries and are unused.
                constexpr int CB = 2;
                constexpr int EO = C::MC + 2;
                // with shifted energies, every slot's shift, the searches of
                // all slots in lockstep (their LDS reads in flight together)
                float dsh_all[LK ? JK : 1];
                if constexpr (LK) {
                    if (shift)
                        on_tables([&](const float *E) { jes_shift_n<JK>(lk_axes(Q, E), E, Q.jd, jpt, jeta, dsh_all); });
                    else
#pragma unroll
                        for (int k = 0; k < JK; ++k) dsh_all[LK ? k : 0] = 0.0f;
                }
                // MS: per slot, whether the jet is a candidate (selected at
                // some scale), a b-tagged candidate, and its shift (LK)
                bool okv[MS ? JK : 1], tagv[MS ? JK : 1];
                float dshv[(MS && LK) ? JK : 1];
#pragma unroll
                for (int k = 0; k < (MS ? JK : 1); ++k) okv[k] = tagv[k] = false;
#pragma unroll
                for (int k0 = 0; k0 < JK; k0 += CB) {
                    if (64 * k0 >= nj) break;  // no jet in this pair or later (uniform)
                    // both slots' range words, then both slots' first two
                    // leptons, each set read together and waited for once (the
                    // pins keep the compiler from moving a read into the
                    // per-slot code)
                    uint32_t pk[CB], pe[CB];
#pragma unroll
                    for (int b = 0; b < CB; ++b) {
                        pk[b] = pe[b] = 0u;
                        if (k0 + b >= JK) continue;
                        pk[b] = L.jr[lane + 64 * (k0 + b)].rng;
                        if (EXT && !C::PACK) pe[b] = L.jre[(EXT && !C::PACK) ? lane + 64 * (k0 + b) : 0];
                    }
                    // (pinned in the extended schema only: the base kernel hides
                    // the latency with more wavefronts and measured faster
                    // with the compiler's own placement)
                    if (EXT) asm volatile("" : "+v"(pk[0]), "+v"(pk[1]));
                    if (EXT && !C::PACK) asm volatile("" : "+v"(pe[0]), "+v"(pe[1]));
                    // per slot: first muon, muon count, offset of the electrons
                    // in the lepton index, lepton count
                    int s0[CB], nmu_[CB], ofe[CB], nlep[CB];
                    float e0[CB], p0[CB], e1[CB], p1[CB];
#pragma unroll
                    for (int b = 0; b < CB; ++b) {
                        const bool live = k0 + b < JK && lane + 64 * (k0 + b) < nj;
                        const uint32_t wm = live ? pk[b] : 0u;
                        const uint32_t we = live ? (C::PACK ? (pk[b] >> 16) : pe[b]) : 0u;
                        s0[b] = static_cast<int>(C::PACK ? (wm & 0xffu) : (wm & 0xffffu));
                        nmu_[b] = static_cast<int>(C::PACK ? ((wm >> 8) & 0xffu) : (wm >> 16));
                        const int u0 = EXT ? static_cast<int>(C::PACK ? (we & 0xffu) : (we & 0xffffu)) : 0;
                        const int nel = EXT ? static_cast<int>(C::PACK ? ((we >> 8) & 0xffu) : (we >> 16)) : 0;
                        ofe[b] = EXT ? EO + u0 - nmu_[b] : s0[b];
                        nlep[b] = nmu_[b] + nel;
                        const int i0 = nmu_[b] >= 1 ? s0[b] : ofe[b];
                        const int i1 = nmu_[b] >= 2 ? s0[b] + 1 : ofe[b] + 1;
                        e0[b] = L.seta[i0];
                        p0[b] = L.sphi[i0];
                        e1[b] = L.seta[i1];
                        p1[b] = L.sphi[i1];
                    }
                    if (EXT)
                        asm volatile("" : "+v"(e0[0]), "+v"(p0[0]), "+v"(e1[0]), "+v"(p1[0]), "+v"(e0[1]),
                                     "+v"(p0[1]), "+v"(e1[1]), "+v"(p1[1]));
#pragma unroll
                    for (int b = 0; b < CB; ++b) {
                        const int k = k0 + b;
                        const int j = lane + 64 * k;
                        if (k >= JK) continue;
                        const bool live = j < nj;
                        // with shifted energies, the jet's shift and the largest
                        // energy it takes over the query's scales
                        const float dsh = shift ? dsh_all[LK ? k : 0] : 0.0f;
                        const float ub = shift ? shifted_pt_bound(jpt[k], dsh, smin, smax) : jpt[k] * smax;
                        const bool need = live & (fabsf(jeta[k]) < jet_abseta) & ((jet_pt < 0.0f) | (ub > jet_pt));
                        const int cn = need ? nlep[b] : 0;
                        bool hit = (cn >= 1 & delta_r2(jeta[k], jphi[k], e0[b], p0[b]) <= thr2) |
                                   (cn >= 2 & delta_r2(jeta[k], jphi[k], e1[b], p1[b]) <= thr2);
                        const int sm = s0[b], nm_ = nmu_[b], oe = ofe[b];
                        auto lidx = [&](int i) { return i < nm_ ? sm + i : oe + i; };
                        int i = 2;
                        // two leptons per step: both LDS reads in flight before the math
                        for (; i + 2 <= cn; i += 2) {
                            const int ia = lidx(i), ib = lidx(i + 1);
                            const float ea = L.seta[ia], pa = L.sphi[ia], eb = L.seta[ib], pb = L.sphi[ib];
                            hit |= delta_r2(jeta[k], jphi[k], ea, pa) <= thr2;
                            hit |= delta_r2(jeta[k], jphi[k], eb, pb) <= thr2;
                        }
                        if (i < cn) {
                            const int ia = lidx(i);
                            hit |= delta_r2(jeta[k], jphi[k], L.seta[ia], L.sphi[ia]) <= thr2;
                        }
                        const bool ok = need && !hit;
                        const bool tag = has_bt && jbt[EXT ? k : 0] > btag;
                        if (MS) {
                            okv[MS ? k : 0] = ok;
                            tagv[MS ? k : 0] = ok && tag;
                            if (LK) dshv[(MS && LK) ? k : 0] = dsh;
                        } else if (!live) {
                        } else if (zsel) {
                            // one scale s (= smax): the jet's energy pt * s, or
                            // pt * (1 + s * d) when shifted
                            const float f = shift ? 1.0f + smax * dsh : smax;
                            L.jr[j].pt = ok ? jpt[k] * f : 0.0f;
                            if (EXT) L.bt[j] = (ok && tag) ? 1 : 0;
                        } else {
                            L.jr[j].pt = ok ? jpt[k] : __builtin_nanf("");
                            if (LK) L.jd[LK ? j : 0] = dsh;
                            if (EXT) L.bt[j] = tag ? 1 : 0;
                        }
                    }
                }
                wave_sync();
                if (MS) {
                    // The candidates -- jets inside |eta|, clean, and (with
                    // jet_pt >= 0) above jet_pt at the largest energy any
                    // scale gives them -- compacted in tile order with their
                    // b-tag flag (and shift).  A jet that is no candidate is
                    // selected at no scale, so walking only the candidates
                    // adds the same values in the same order.  cpre gives
                    // every event its candidate range and, with jet_pt >= 0,
                    // its candidate and b-tagged candidate counts: the jets
                    // selected and b-tagged at the largest scale.
                    int runc = 0, runt = 0;
#pragma unroll
                    for (int k = 0; k < JK; ++k) {
                        if (64 * k >= nj) break;
                        const int j = lane + 64 * k;
                        const uint64_t bc = __ballot(okv[MS ? k : 0]), bg = __ballot(tagv[MS ? k : 0]);
                        const int before = runc + static_cast<int>(__builtin_amdgcn_mbcnt_hi(
                                                      static_cast<uint32_t>(bc >> 32),
                                                      __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(bc), 0u)));
                        const int tbefore = runt + static_cast<int>(__builtin_amdgcn_mbcnt_hi(
                                                       static_cast<uint32_t>(bg >> 32),
                                                       __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(bg), 0u)));
                        if (j < nj) L.cpre[MS ? j : 0] = static_cast<uint32_t>(before) | (static_cast<uint32_t>(tbefore) << 16);
                        if (okv[MS ? k : 0]) {
                            L.jr[before].pt = jpt[k];
                            if (EXT) L.bt[before] = tagv[MS ? k : 0] ? 1 : 0;
                            if (LK) L.jd[LK ? before : 0] = dshv[(MS && LK) ? k : 0];
                        }
                        runc += __popcll(bc);
                        runt += __popcll(bg);
                    }
                    if (lane == 0) L.cpre[MS ? nj : 0] = static_cast<uint32_t>(runc) | (static_cast<uint32_t>(runt) << 16);
                    wave_sync();
                    // the tile's columns are dead from here on: the next
                    // tile's loads can fly during this query's walk and fills
                    if (q == qlast) after_cone();
                }
                // ---- 5. per-event reductions, event cut, fills
                const FillC F = fill_consts<LDSH, MS>(Q);
                // separate calls for the two places the edges live, so each
                // knows its address space (no flat loads)
                const int vlast = Q.n_scale - 1;
                auto fill = [&](const auto &xs, const auto &pass, int v0, double w) {
                    constexpr int N = std::extent<std::remove_reference_t<decltype(xs)>>::value;
                    if (P.edges_in_lds)
                        fill_bins<N, MS>(sink, F, e_s, xs, pass, v0, w, vlast);
                    else
                        fill_bins<N, MS>(sink, F, P.edges, xs, pass, v0, w, vlast);
                };
                if (!MS) {
                    const float sc[1] = {pin<float>(as_const(P.scales)[Q.scale0])};
#pragma unroll
                    for (int r = 0; r < EVPL; ++r) {
                        // an event short of muons or of jets before any cut
                        // cannot pass: its walk is skipped
                        const bool elig = lane + 64 * r < ne && nmu[r] >= min_mu && je[r] - jb[r] >= min_jet;
                        float ht[1], lead[1];
                        int njs[1], nbt[1];
                        const int jend = elig ? je[r] : jb[r];
                        if (zsel)
                            walk_selected<EXT>(L, jb[r], jend, ht[0], lead[0], njs[0], nbt[0]);
                        else if (shift)
                            walk_jets<1, EXT, true>(L, jb[r], jend, sc, jet_pt, ht, lead, njs, nbt);
                        else
                            walk_jets<1, EXT, false>(L, jb[r], jend, sc, jet_pt, ht, lead, njs, nbt);
                        const bool pass[1] = {elig && njs[0] >= min_jet && nbt[0] >= min_b};
                        if (DBG && lane + 64 * r < ne)
                            *rec_at(P, Q.scale0, D.ev0 + e0 + lane + 64 * r) = hepk_event_record{
                                nmu[r], njs[0], nbt[0], elig ? (pass[0] ? 3 : 2) : 1, ht[0], lead[0], wq[r], 0};
                        if (pass[0]) {
                            const float xs[3] = {ht[0], lead[0], static_cast<float>(njs[0])};
                            fill(xs, pass, 0, static_cast<double>(wq[r]));
                        }
                    }
                } else {
                    // Several scales: the events that can pass at some scale are
                    // compacted, and lanes take (event, group of kG scales)
                    // pairs of them, event-major.  One walk over an event's
                    // candidate jets serves the kG scales of its group (kG
                    // independent chains), and a round covers a few events, so
                    // the walks diverge little.  An event can pass only with
                    // enough muons and enough jets before any cut (the cuts
                    // only remove jets); with jet_pt >= 0 also only with
                    // enough selected jets and b-tagged jets at the largest
                    // scale: a jet selected at s <= smax is selected at smax
                    // (rounding pt * s is monotone in s for pt >= 0, and
                    // pt * s <= 0 <= jet_pt otherwise; with shifts, the
                    // largest energy is at smin or smax), and those counts
                    // are the event's candidates and b-tagged candidates.
                    const bool prefilter = jet_pt >= 0.0f;
                    int nel = 0;
#pragma unroll
                    for (int r = 0; r < EVPL; ++r) {
                        const uint32_t cw0 = L.cpre[MS ? jb[r] : 0], cw1 = L.cpre[MS ? je[r] : 0];
                        const int cb = static_cast<int>(cw0 & 0xffffu), ce = static_cast<int>(cw1 & 0xffffu);
                        bool elig = lane + 64 * r < ne && nmu[r] >= min_mu && je[r] - jb[r] >= min_jet;
                        if (prefilter)
                            elig = elig && ce - cb >= min_jet && static_cast<int>((cw1 >> 16) - (cw0 >> 16)) >= min_b;
                        if (DBG && lane + 64 * r < ne) {
                            // the muon count of every event; the rest only of
                            // events that are not walked (the walk writes the
                            // other fields of walked events' records)
                            const int64_t ge = D.ev0 + e0 + lane + 64 * r;
                            for (int v = 0; v < Q.n_scale; ++v) {
                                hepk_event_record *o = rec_at(P, Q.scale0 + v, ge);
                                o->n_mu = nmu[r];
                                o->w = wq[r];
                                o->reserved = 0;
                                if (!elig) {
                                    o->n_jet = 0;
                                    o->n_b = 0;
                                    o->state = 1;
                                    o->ht = 0.0f;
                                    o->lead = -INFINITY;
                                }
                            }
                        }
                        const uint64_t bal = __ballot(elig);
                        const int at = nel + static_cast<int>(__builtin_amdgcn_mbcnt_hi(
                                                 static_cast<uint32_t>(bal >> 32),
                                                 __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(bal), 0u)));
                        if (elig) {
                            // candidate range: first in bits 0-9, end in bits
                            // 16-25 (both at most 64 * JK <= 832); DBG kernels
                            // keep the event's place in the tile in the bits
                            // between
                            const uint32_t ev = static_cast<uint32_t>(lane + 64 * r);
                            L.u.w.evjr[at] = static_cast<uint32_t>(cb) | (static_cast<uint32_t>(ce) << 16) |
                                             (DBG ? (((ev & 63u) << 10) | ((ev >> 6) << 26)) : 0u);
                            L.u.w.evw[at] = wq[r];
                        }
                        nel += __popcll(bal);
                    }
                    wave_sync();
                    int V = Q.n_scale, scale0 = Q.scale0;
                    asm volatile("" : "+s"(V), "+s"(scale0));
                    const float *scl = (P.scales_in_lds ? s_s : P.scales) + scale0;
                    const int NG = (V + kG - 1) / kG;
                    const int npairs = nel * NG;
                    int e = lane / NG, g = lane - (lane / NG) * NG;
                    const int de = 64 / NG, dg = 64 - (64 / NG) * NG;
                    for (int i = lane; i < npairs; i += 64) {
                        const uint32_t jr = L.u.w.evjr[e];
                        float sc[kG];
#pragma unroll
                        for (int u = 0; u < kG; ++u) sc[u] = scl[min(g * kG + u, V - 1)];
                        float ht[kG], lead[kG];
                        int njs[kG], nbt[kG];
                        const int wj0 = static_cast<int>(jr & 0x3ffu), wj1 = static_cast<int>((jr >> 16) & 0x3ffu);
                        if (shift)
                            walk_jets<kG, EXT, true>(L, wj0, wj1, sc, jet_pt, ht, lead, njs, nbt);
                        else
                            walk_jets<kG, EXT, false>(L, wj0, wj1, sc, jet_pt, ht, lead, njs, nbt);
                        bool pass[kG], any = false;
#pragma unroll
                        for (int u = 0; u < kG; ++u) {
                            pass[u] = g * kG + u < V && njs[u] >= min_jet && nbt[u] >= min_b;
                            any |= pass[u];
                        }
                        if (DBG) {
                            const int64_t ge = D.ev0 + e0 + (((jr >> 10) & 63u) | ((jr >> 26) << 6));
#pragma unroll
                            for (int u = 0; u < kG; ++u) {
                                if (g * kG + u >= V) continue;
                                hepk_event_record *o = rec_at(P, scale0 + g * kG + u, ge);
                                o->n_jet = njs[u];
                                o->n_b = nbt[u];
                                o->state = pass[u] ? 3 : 2;
                                o->ht = ht[u];
                                o->lead = lead[u];
                            }
                        }
                        if (any) {
                            // FS scales' bins per search: the batch that fits the
                            // registers of 1024-thread workgroups without spilling
                            // (one while the next tile's loads are in flight)
                            constexpr int FS = PIPE ? 1 : 2;
                            const double w = static_cast<double>(L.u.w.evw[e]);
#pragma unroll
                            for (int u = 0; u < kG; u += FS) {
                                float xs[3 * FS];
                                bool pu[FS], anyu = false;
#pragma unroll
                                for (int t = 0; t < FS; ++t) {
                                    xs[3 * t] = ht[u + t];
                                    xs[3 * t + 1] = lead[u + t];
                                    xs[3 * t + 2] = static_cast<float>(njs[u + t]);
                                    pu[t] = pass[u + t];
                                    anyu |= pu[t];
                                }
                                if (anyu) fill(xs, pu, g * kG + u, w);
                            }
                        }
                        e += de;
                        g += dg;
                        if (g >= NG) {
                            g -= NG;
                            e += 1;
                        }
                    }
                }
                wave_sync();
            }
        };
        // Tile bounds are fetched one tile ahead (scalar loads that overlap
        // the current tile's vector loads).  A tile whose objects exceed the
        // register capacity runs as consecutive sub-tiles: from its first
        // event not yet run, the event count is halved until the objects fit
        // (a few scalar loads), that sub-tile runs like a tile, and the rest
        // of the tile follows.  Only a single event beyond the capacity goes
        // one lane, straight from HBM.  With several scales (PIPE) the next
        // (sub-)tile's loads are issued into R as soon as the last query's
        // cone test is done, so they are in flight during the walks and fills.
        int r = wave;  // this wavefront's tile (relative to c_t0)
        int eo = 0;    // events of tile r already run
        TileBounds nb{};
        if (r < nt) nb = bounds_of(r);
        Raw R;
        bool have = false;  // R already holds the loads of the current (sub-)tile
        while (r < nt) {
            // the lane index is re-read here so that values derived from it
            // are recomputed per tile instead of held (and spilled) across it
            asm volatile("" : "+v"(lane));
            const int tn = tile_events(r);
            const int64_t e = ebase + static_cast<int64_t>(r) * TW + eo;
            int n = tn - eo;
            TileBounds B;
            if (eo == 0) {
                B = nb;
                if (r + WAVES < nt) nb = bounds_of(r + WAVES);
            } else {
                B = tile_bounds<EXT>(D, has_el, e, n);
            }
            while (n > 1 && oversize(B)) {
                n = (n + 1) >> 1;
                B = tile_bounds<EXT>(D, has_el, e, n);
            }
            // the position after this (sub-)tile; nb holds the bounds of
            // tile r + WAVES whenever it starts a tile
            int r2 = r, eo2 = eo + n;
            if (eo2 >= tn) {
                r2 = r + WAVES;
                eo2 = 0;
            }
            if (oversize(B)) {
                const DsDev Dc = D;
                if (lane == 0) event_direct<T, EXT, LDSH, DBG, LK>(P, Dc, e, edges, sink);
                have = false;
            } else {
                if (!have) issue(e, n, B, R);
                settle(R);
                bool issued = false;
                auto next_loads = [&]() {
                    if (!PIPE || r2 >= nt) return;
                    const int64_t e2 = ebase + static_cast<int64_t>(r2) * TW + eo2;
                    int n2 = tile_events(r2) - eo2;
                    TileBounds B2 = eo2 == 0 ? nb : tile_bounds<EXT>(D, has_el, e2, n2);
                    while (n2 > 1 && oversize(B2)) {
                        n2 = (n2 + 1) >> 1;
                        B2 = tile_bounds<EXT>(D, has_el, e2, n2);
                    }
                    if (oversize(B2)) return;
                    issue(e2, n2, B2, R);
                    issued = true;
                };
                work(e, n, B, R, next_loads);
                have = issued;
            }
            r = r2;
            eo = eo2;
        }
        // merge the LDS histograms into the dataset's block in HBM (the next
        // chunk, if any, is another dataset)
        if (LDSH) {
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
                                if (LK && P.sumw2) atomic_add_f64(&P.sumw2[gs + i], sw2_s[ls + i]);
                                c_s[ls + i] = 0u;
                                sw_s[ls + i] = 0.0;
                                if (LK) sw2_s[ls + i] = 0.0;
                            }
                        }
                    }
            }
            __syncthreads();
        }
    }
}

using KernelFn = void (*)(PipeArgs);

template <typename T, bool EXT, int WAVES, int EVPL, bool LDSH, bool MS, bool DBG, bool LK>
static KernelFn kfn() {
    return reinterpret_cast<KernelFn>(&pipeline_kernel<T, EXT, WAVES, EVPL, LDSH, MS, DBG, LK>);
}

template <typename T, bool EXT, int WAVES, int EVPL, bool MS, bool DBG, bool LK>
static KernelFn pick_h(bool ldsh) {
    return ldsh ? kfn<T, EXT, WAVES, EVPL, true, MS, DBG, LK>() : kfn<T, EXT, WAVES, EVPL, false, MS, DBG, LK>();
}

// LK kernels exist for one event per thread only (the plan takes that shape
// for queries with lookups).
template <typename T, bool EXT, bool MS, bool DBG, bool LK>
static KernelFn pick_shape(int block, int evpt, bool ldsh) {
    if (block == 1024) return pick_h<T, EXT, 16, 1, MS, DBG, LK>(ldsh);  // one event per thread only
    if (LK) return block == 512 ? pick_h<T, EXT, 8, 1, MS, DBG, LK>(ldsh) : pick_h<T, EXT, 4, 1, MS, DBG, LK>(ldsh);
    if (block == 512)
        return evpt == 2 ? pick_h<T, EXT, 8, 2, MS, DBG, LK>(ldsh) : pick_h<T, EXT, 8, 1, MS, DBG, LK>(ldsh);
    return evpt == 2 ? pick_h<T, EXT, 4, 2, MS, DBG, LK>(ldsh) : pick_h<T, EXT, 4, 1, MS, DBG, LK>(ldsh);
}

// The kernel for a launch shape; each (MS, DBG, LK) triple is instantiated
// in its own translation unit (they compile in parallel).
template <bool MS, bool DBG, bool LK>
KernelFn pick_kernel(int dtype, bool ext, int block, int evpt, bool ldsh) {
    if (dtype == HEPK_F16) return ext ? pick_shape<_Float16, true, MS, DBG, LK>(block, evpt, ldsh)
                                      : pick_shape<_Float16, false, MS, DBG, LK>(block, evpt, ldsh);
    return ext ? pick_shape<float, true, MS, DBG, LK>(block, evpt, ldsh)
               : pick_shape<float, false, MS, DBG, LK>(block, evpt, ldsh);
}

// LDS for the workgroup's private histograms: up to 144 KiB (60 histograms of
// 100 bins with squared weights fit), as long as the workgroup's total fits
// the device; larger sets go to global atomics.  More LDS lowers occupancy,
// which the launch-configuration search weighs against atomic contention.
constexpr int kMaxLdsHistBytes = 144 * 1024;
constexpr int kMaxLdsEdgeBytes = 4 * 1024;
constexpr int kMaxLdsScaleBytes = 1024;

}  // namespace hepk
