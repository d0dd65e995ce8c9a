// gfx950 kernels of the Heisenberg Pauli-propagation hot path.
//
// Layout: the live operator is kept sorted by (X, z), X being the x mask stored
// rotated right by the number of sigma_x rotations applied so far in the
// current layer, so that the qubit of the next RX gate always sits at stored
// bit 0.  For a sigma_x generator on that qubit, a string and its partner
// I xor J differ in stored bit 0 only: they lie in two adjacent x-groups
// (the "A" group with bit 0 clear and the "B" group with bit 0 set) of one
// pairing block, at the same z.  One gate (Eq. update_rule, Algorithm 1 gate
// loop + apply-received loop) is therefore a merge by z of the two groups of
// every block; the outputs with x_j = 0 go to the front run of the output
// buffer and those with x_j = 1 to its back run, which yields the next gate's
// order (stored x rotated by one more bit) without any sort.
#include "orqa_device.h"

namespace orqa {

// ================================================================ RX: tile split
// Sorted order of the input: (X, z).  A pairing block = equal X with bit 0
// cleared.  Merged order inside a block: by z, A before B on ties, so a
// string and its partner are adjacent.  Merging permutes strings only inside
// their block, so merged position b and input position b lie in the same
// block; tile t covers merged positions [t kRxTile, (t+1) kRxTile), its
// boundaries moved by one where they would separate a pair.

struct VIn {
    const ulonglong2* X;
    const ulonglong2* Z;
    uint64_t nf, cap;
    __device__ __forceinline__ ulonglong2 x(uint64_t i) const { return X[vphys(i, nf, cap)]; }
    __device__ __forceinline__ ulonglong2 z(uint64_t i) const { return Z[vphys(i, nf, cap)]; }
};

// First index in [lo, hi) where pred holds, hi if none; pred must be
// monotone in the index (false ... false true ... true).  Called by all 64
// lanes of a wave with uniform bounds: each round probes 64 evenly spaced
// indices and shrinks the range 64-fold, so a range of up to 64 takes one
// round trip to memory.
template <class Pred>
__device__ __forceinline__ uint64_t wave_lower_bound(uint64_t lo, uint64_t hi, Pred pred) {
    const uint64_t lane = uint64_t(lane_id());
    while (lo < hi) {
        const uint64_t step = (hi - lo + 63) >> 6;
        const uint64_t q = lo + (lane + 1) * step - 1;
        const uint64_t bal = __ballot(q >= hi || pred(q));
        if (bal == 0) return hi;  // then lane 63 probed hi - 1
        const uint64_t L = uint64_t(__ffsll(static_cast<unsigned long long>(bal)) - 1);
        const uint64_t qL = lo + (L + 1) * step - 1;
        lo += L * step;
        if (qL < hi) hi = qL;
    }
    return lo;
}

// The same split by one thread (binary searches; few registers, many
// dependent loads): the fallback of a tile whose boundaries were not found in
// time by the grid.
__device__ uint64_t first_geq_h(const VIn& v, ulonglong2 key, uint64_t lo, uint64_t hi, bool strict) {
    while (lo < hi) {  // first i in [lo, hi) with h(X[i]) >= key (> key when strict)
        const uint64_t mid = lo + (hi - lo) / 2;
        const ulonglong2 h = k_h(v.x(mid));
        if (strict ? k_le(h, key) : k_lt(h, key)) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ TileDesc thread_split(const VIn& v, uint64_t n, uint64_t b) {
    if (b >= n) return {n, n, n, n};
    const ulonglong2 H = k_h(v.x(b));
    const uint64_t hs = first_geq_h(v, H, 0, b, false);
    const uint64_t he = first_geq_h(v, H, b + 1, n, true);
    uint64_t lo = hs, hi = he;  // first B string: first X >= (H with bit 0 set)
    const ulonglong2 H1 = make_ulonglong2(H.x | 1ull, H.y);
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (k_lt(v.x(mid), H1)) lo = mid + 1;
        else hi = mid;
    }
    const uint64_t hm = lo, na = hm - hs, nbb = he - hm, d = b - hs;
    uint64_t ilo = d > nbb ? d - nbb : 0, ihi = d < na ? d : na;
    while (ilo < ihi) {
        const uint64_t mid = ilo + (ihi - ilo) / 2;
        if (k_le(v.z(hs + mid), v.z(hm + d - 1 - mid))) ilo = mid + 1;
        else ihi = mid;
    }
    uint64_t k = d - ilo;
    if (ilo > 0 && k < nbb && k_eq(v.z(hs + ilo - 1), v.z(hm + k))) k += 1;
    return {hs + ilo, hm + k, hm, he};
}

__device__ __forceinline__ ulonglong2 shfl_u128(const ulonglong2& v, int src) {
    const uint32_t a = __shfl(static_cast<uint32_t>(v.x), src, 64);
    const uint32_t b = __shfl(static_cast<uint32_t>(v.x >> 32), src, 64);
    const uint32_t c = __shfl(static_cast<uint32_t>(v.y), src, 64);
    const uint32_t d = __shfl(static_cast<uint32_t>(v.y >> 32), src, 64);
    return make_ulonglong2((uint64_t(b) << 32) | a, (uint64_t(d) << 32) | c);
}

// Split of merged position b (all 64 lanes, uniform result): the input
// positions where it falls in the A and B groups of its pairing block, the
// block's first B position and its end.  One window of 128 keys around b
// (one round trip to memory) settles any block that lies inside it, the
// merge path included; wider blocks take 64-ary searches.
// Ends of a pairing block wider than the split window (all 64 lanes, uniform
// H): the block start hs = first i <= b - 64 with h(x_i) >= H when need_s
// (the window's back half lies inside the block), and the block end he =
// first i >= b + 64 with h(x_i) > H when need_e.  Lanes 0-31 look backwards
// from b - 64 and lanes 32-63 forwards from b + 63, at 16 distances 32 apart
// and then 16 doubling ones (one round trip for both ends), then each half
// narrows its bracket by 32-ary search.
__device__ void block_ends(const VIn& v, uint64_t n, uint64_t b, const ulonglong2& H, bool need_s, bool need_e,
                           uint64_t& hs, uint64_t& he) {
    const int lane = lane_id();
    const bool fwd = lane >= 32;
    const int l = lane & 31;
    const bool need = fwd ? need_e : need_s;
    auto dist = [](int j) { return j < 16 ? 32ull * uint64_t(j + 1) : (512ull << (j - 15)); };
    // probe j of the back half is b - 64 - dist(j), of the front half b + 63 + dist(j);
    // "outside" = before the block (back) or after it (front), positions
    // beyond the operator included
    bool out = true;
    if (need) {
        if (!fwd) {
            const int64_t q = int64_t(b) - 64 - int64_t(dist(l));
            out = q < 0 || k_lt(k_h(v.x(uint64_t(q))), H);
        } else {
            const uint64_t q = b + 63 + dist(l);
            out = q >= n || k_lt(H, k_h(v.x(q)));
        }
    }
    const uint64_t bal0 = __ballot(out);
    const uint32_t ob = uint32_t(fwd ? (bal0 >> 32) : bal0);
    // bracket [lo, hi): the answer is the first position in it where the
    // predicate holds, hi if none (the predicate holds at hi)
    uint64_t lo = 0, hi = 0;
    if (need) {
        const int L = ob ? __ffs(ob) - 1 : 32;  // first probe outside; 32: none
        if (!fwd) {
            const int64_t qin = L == 0 ? int64_t(b) - 64 : int64_t(b) - 64 - int64_t(dist(L - 1));
            const int64_t qout = L < 32 ? int64_t(b) - 64 - int64_t(dist(L)) : -1;
            lo = qout < 0 ? 0 : uint64_t(qout + 1);
            hi = uint64_t(qin);
        } else {
            const uint64_t qin = L == 0 ? b + 63 : b + 63 + dist(L - 1);
            const uint64_t qout = L < 32 ? b + 63 + dist(L) : n;
            lo = qin + 1;
            hi = qout < n ? qout : n;
        }
    }
    for (;;) {
        const bool act = need && lo < hi;
        if (__ballot(act) == 0) break;
        const uint64_t step = act ? (hi - lo + 31) >> 5 : 1;
        const uint64_t q = lo + uint64_t(l + 1) * step - 1;
        bool pr = false;
        if (act) pr = q >= hi || (fwd ? k_lt(H, k_h(v.x(q))) : !k_lt(k_h(v.x(q)), H));
        const uint64_t bal = __ballot(pr);
        const uint32_t hb = uint32_t(fwd ? (bal >> 32) : bal);
        if (act) {
            if (hb == 0) {
                lo = hi;
            } else {
                const uint64_t L2 = uint64_t(__ffs(hb) - 1);
                const uint64_t qL = lo + (L2 + 1) * step - 1;
                lo += L2 * step;
                if (qL < hi) hi = qL;
            }
        }
    }
    const uint64_t r_s = __shfl(lo, 0), r_e = __shfl(lo, 32);
    if (need_s) hs = r_s;
    if (need_e) he = r_e;
}

struct SplitWin {
    ulonglong2 xb, xf, zb, zf;  // lane l: keys at b - 64 + l and b + l (lane 0's second key is b)
};

__device__ __forceinline__ SplitWin split_window(const VIn& v, uint64_t n, uint64_t b) {
    const int lane = lane_id();
    const int64_t pb = int64_t(b) - 64 + lane;
    const uint64_t pf = b + uint64_t(lane);
    SplitWin w;
    w.xb = pb >= 0 ? v.x(uint64_t(pb)) : make_ulonglong2(0, 0);
    w.xf = pf < n ? v.x(pf) : make_ulonglong2(0, 0);
    w.zb = pb >= 0 ? v.z(uint64_t(pb)) : make_ulonglong2(0, 0);
    w.zf = pf < n ? v.z(pf) : make_ulonglong2(0, 0);
    return w;
}

// b < n; W is split_window(v, n, b)
__device__ TileDesc wave_split_win(const VIn& v, uint64_t n, uint64_t b, const SplitWin& W) {
    const int lane = lane_id();
    const int64_t pb = int64_t(b) - 64 + lane;
    const uint64_t pf = b + uint64_t(lane);
    const ulonglong2 xb = W.xb, xf = W.xf, zb = W.zb, zf = W.zf;
    const ulonglong2 H = k_h(shfl_u128(xf, 0));
    const ulonglong2 H1 = make_ulonglong2(H.x | 1ull, H.y);
    // block start: h is non-decreasing, so the lanes before the block form a prefix
    const uint64_t before = __ballot(pb < 0 || k_lt(k_h(xb), H));
    // block end (lane 0 reads b itself, which is inside)
    const uint64_t after = __ballot(pf >= n || k_lt(H, k_h(xf)));
    uint64_t hs = 0, he = 0;
    if (before != 0) hs = uint64_t(int64_t(b) - 64 + __popcll(before));
    if (after != 0) he = b + uint64_t(__ffsll(static_cast<unsigned long long>(after)) - 1);
    if (before == 0 || after == 0) block_ends(v, n, b, H, before == 0, after == 0, hs, he);
    // first B string of the block: exact when the window holds both an A and
    // a B string of the block, else searched beyond the window's B (or A) part
    const uint64_t mb = __ballot(pb >= int64_t(hs) && !k_lt(xb, H1));
    const uint64_t mf = __ballot(pf < he && !k_lt(xf, H1));
    const uint64_t ab = __ballot(pb >= int64_t(hs) && k_lt(xb, H1));
    const uint64_t af = __ballot(pf < he && k_lt(xf, H1));
    const bool hasB = (mb | mf) != 0, hasA = (ab | af) != 0;
    uint64_t bfirst = he, alast = hs;  // first B and one past the last A in the window
    if (hasB) bfirst = mb ? uint64_t(int64_t(b) - 64 + (__ffsll(static_cast<unsigned long long>(mb)) - 1))
                          : b + uint64_t(__ffsll(static_cast<unsigned long long>(mf)) - 1);
    if (hasA) alast = af ? b + uint64_t(63 - __clzll(af)) + 1
                         : uint64_t(int64_t(b) - 64 + (63 - __clzll(ab))) + 1;
    uint64_t hm;
    if ((before != 0 && after != 0) || (hasA && hasB)) {
        hm = hasB ? bfirst : he;  // the window covers the A-to-B change
    } else {
        hm = wave_lower_bound(hasA ? alast : hs, hasB ? bfirst : he,
                              [&](uint64_t i) { return !k_lt(v.x(i), H1); });
    }
    const uint64_t na = hm - hs, nbb = he - hm, d = b - hs;
    // merge path: i = number of A strings among the first d merged
    const uint64_t ilo = d > nbb ? d - nbb : 0, ihi = d < na ? d : na;
    uint64_t i;
    ulonglong2 za, zk;  // z of A string i - 1 and of B string k (the pair check)
    uint64_t k;
    if (before != 0 && after != 0) {
        // the whole block is in the window: z of position p from the lane
        // that read it (ihi - ilo <= d <= 64, so one probe per lane)
        auto zwin = [&](uint64_t p) {
            const bool back = p < b;
            const int src = back ? int(int64_t(p) - (int64_t(b) - 64)) : int(p - b);
            const ulonglong2 u = shfl_u128(zb, src), w2 = shfl_u128(zf, src);
            return back ? u : w2;
        };
        const uint64_t mid = ilo + uint64_t(lane);
        const uint64_t pa = hs + (mid < ihi ? mid : ilo);
        const uint64_t pq = hm + d - 1 - (mid < ihi ? mid : ilo);
        const ulonglong2 zA = zwin(pa < he ? pa : hs), zB = zwin(pq < he ? pq : hs);
        const uint64_t bal = __ballot(mid < ihi && !k_le(zA, zB));
        i = (ilo < ihi && bal != 0) ? ilo + uint64_t(__ffsll(static_cast<unsigned long long>(bal)) - 1) : ihi;
        k = d - i;
        const uint64_t p1 = i > 0 ? hs + i - 1 : hs, p2 = hm + k < he ? hm + k : hs;
        za = zwin(p1);
        zk = zwin(p2);
    } else {
        i = wave_lower_bound(ilo, ihi,
                             [&](uint64_t m) { return !k_le(v.z(hs + m), v.z(hm + d - 1 - m)); });
        k = d - i;
        za = v.z(i > 0 ? hs + i - 1 : hs);
        zk = v.z(hm + k < he ? hm + k : hs);
    }
    if (i > 0 && k < nbb && k_eq(za, zk)) k += 1;  // keep the pair together
    return {hs + i, hm + k, hm, he};
}

__device__ TileDesc wave_split(const VIn& v, uint64_t n, uint64_t b) {
    if (b >= n) return {n, n, n, n};
    return wave_split_win(v, n, b, split_window(v, n, b));
}

// Tile boundaries of an RX gate's input, found by the merge kernel itself
// before it takes tiles: wave w of the grid finds boundaries w, w + W, ...
// (W waves), the split of merged position t kRxTile for t = 0 .. ntiles (the
// last one at n).  Each of its four words is stored as a status word of the
// launch's epoch, so a tile reads its two boundaries as soon as they are
// there, with no fence and no grid-wide wait.
struct TileDescWords {
    uint64_t w[4];  // posA, posB, hm, he, each tagged like a look-back status word
};

__device__ __forceinline__ void rx_boundaries(const VIn& v, uint64_t n, TileDescWords* desc, uint32_t ep) {
    const uint64_t ntiles = (n + kRxTile - 1) / kRxTile;
    const uint64_t waves = uint64_t(gridDim.x) * (kThreads / 64);
    uint64_t t = blockIdx.x * uint64_t(kThreads / 64) + (threadIdx.x >> 6);
    if (t > ntiles) return;
    // the window of the wave's next boundary is in flight while this one is settled
    SplitWin w = split_window(v, n, t * kRxTile < n ? t * kRxTile : n);
    for (; t <= ntiles; t += waves) {
        const uint64_t b = t * kRxTile < n ? t * kRxTile : n;
        const uint64_t tn = t + waves;
        SplitWin wn = w;
        if (tn <= ntiles) wn = split_window(v, n, tn * kRxTile < n ? tn * kRxTile : n);
        const TileDesc d = b < n ? wave_split_win(v, n, b, w) : TileDesc{n, n, n, n};
        w = wn;
        const int lane = lane_id();
        if (lane < 4) {
            const uint64_t val = lane == 0 ? d.posA : lane == 1 ? d.posB : lane == 2 ? d.hm : d.he;
            st_rel(&desc[t].w[lane], st_pack(ep, 2, val));
        }
    }
}

// The boundaries of tiles t and t + 1 (uniform), read by wave 0 once all
// eight words carry this launch's epoch and handed to the workgroup through
// s_desc (two entries of LDS).  Boundaries that have not arrived after
// kDescWaitTicks are found by the workgroup itself (waves 0 and 1) and
// published: a tile never depends on a workgroup that is not running yet.
constexpr uint64_t kDescWaitTicks = 3000;  // 30 us of the 100 MHz wall clock

__device__ __forceinline__ void rx_read_boundaries(const VIn& v, uint64_t n, TileDescWords* desc, uint64_t t,
                                                   uint32_t ep, TileDesc* s_desc, uint32_t* s_flag) {
    if ((threadIdx.x >> 6) == 0) {
        const int lane = lane_id();
        const uint64_t t0 = wall_clock64();
        uint64_t w = 0;
        bool ready = false;
        while (true) {
            if (lane < 8) w = ld_acq(&desc[t + (lane >> 2)].w[lane & 3]);
            if (!__any(lane < 8 && st_flag(w, ep) != 2u)) {
                ready = true;
                break;
            }
            if (__any(wall_clock64() - t0 > kDescWaitTicks)) break;
            __builtin_amdgcn_s_sleep(kLb2Sleep);
        }
        if (lane < 8) reinterpret_cast<uint64_t*>(s_desc)[lane] = w & kValMask;
        if (lane == 0) *s_flag = ready ? 1u : 0u;
    }
    __syncthreads();
    if (*s_flag == 0u) {
        if (threadIdx.x < 2) {
            const uint64_t b = (t + threadIdx.x) * kRxTile;
            const TileDesc d = thread_split(v, n, b < n ? b : n);
            s_desc[threadIdx.x] = d;
            st_rel(&desc[t + threadIdx.x].w[0], st_pack(ep, 2, d.posA));
            st_rel(&desc[t + threadIdx.x].w[1], st_pack(ep, 2, d.posB));
            st_rel(&desc[t + threadIdx.x].w[2], st_pack(ep, 2, d.hm));
            st_rel(&desc[t + threadIdx.x].w[3], st_pack(ep, 2, d.he));
        }
        __syncthreads();
    }
}

// ================================================================ RX: merge
template <typename CT, int LP>
__device__ __forceinline__ bool keep_row(const CT* c, const double* thr) {
    bool keep = false;
#pragma unroll
    for (int a = 0; a < LP; ++a) keep |= absd(c[a]) > thr[a];
    return keep;
}

// Input ranges of one RX tile (uniform across the workgroup).
struct RxTile {
    uint64_t r1s, r2s, r3s;
    uint32_t l1, l2, l3, m;
    bool sane;
};

__device__ __forceinline__ uint64_t uni64(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// Tile ranges from the descriptors of its two boundaries (uniform values,
// kept in scalar registers).
__device__ __forceinline__ RxTile rx_tile(const TileDesc& e0, const TileDesc& e1, uint64_t n) {
    const TileDesc d0{uni64(e0.posA), uni64(e0.posB), uni64(e0.hm), uni64(e0.he)};
    const TileDesc d1{uni64(e1.posA), uni64(e1.posB), uni64(e1.hm), uni64(e1.he)};
    const bool same = (d0.hm == d1.hm) && (d0.he == d1.he);
    const uint64_t r1s = d0.posA, r1e = same ? d1.posA : d0.hm;
    const uint64_t r2s = d0.posB, r2e = same ? d1.posB : d1.posA;
    const uint64_t r3s = same ? 0 : d1.hm, r3e = same ? 0 : d1.posB;
    RxTile t;
    t.sane = r1s <= r1e && r2s <= r2e && r3s <= r3e && r1e <= n && r2e <= n && r3e <= n &&
             (r1e - r1s) + (r2e - r2s) + (r3e - r3s) <= uint64_t(kRxTileMax);
    t.r1s = r1s;
    t.r2s = r2s;
    t.r3s = r3s;
    t.l1 = t.sane ? uint32_t(r1e - r1s) : 0u;
    t.l2 = t.sane ? uint32_t(r2e - r2s) : 0u;
    t.l3 = t.sane ? uint32_t(r3e - r3s) : 0u;
    t.m = t.l1 + t.l2 + t.l3;
    return t;
}

__device__ __forceinline__ uint64_t rx_phys(const RxTile& t, uint32_t e, uint64_t nf, uint64_t cap) {
    const uint64_t li = e < t.l1 ? t.r1s + e : (e < t.l1 + t.l2 ? t.r2s + (e - t.l1) : t.r3s + (e - t.l1 - t.l2));
    return vphys(li, nf, cap);
}

// Output entry of an RX tile: source string e, partner e2 and kind.
//   kind 0: copy c_e; 1: cos * c_e; 2: child sin * c_e (sign by side);
//   kind 3: pair cos * c_e + sin * c_e2 (sign by side)
// Front side (x_j = 0 after the gate) takes the child of a Y partner with the
// minus sign, the back side the child of a Z partner with the plus sign.
__device__ __forceinline__ uint32_t out_entry(uint32_t e, uint32_t e2, uint32_t kind) {
    return e | (e2 << 10) | (kind << 20);
}

template <typename CT, int LP>
__device__ __forceinline__ CT rx_value(const GateTrig& g, int a, uint32_t kind, bool neg, CT ce, CT ce2) {
    if (kind == 0) return ce;
    if (kind == 1) return Arith<CT>::scale_c(g, a, ce);
    if (kind == 2) return Arith<CT>::scale_s(g, a, ce, neg);
    return Arith<CT>::pair(g, a, ce, ce2, neg);
}

constexpr uint32_t kNoTile = 0xFFFFFFFFu;
constexpr int kRxBatch = 2;  // 16-byte chunks per thread whose loads a wide-row loop issues together

// One RX gate, software-pipelined over the tiles a workgroup takes: a tile is
// loaded and planned (x-groups, merged order, emission plan, output counts),
// its output counts published, and its outputs gathered into registers; they
// are written one iteration later, once the look-back has resolved the
// tile's output offsets, so the wait for those offsets overlaps the loading
// and planning of the next tile.  The split descriptors of the next tile are
// found by two waves during the same wait.  A tile with more outputs than
// the registers hold (KR per thread) is resolved and written at once; with
// KR = 0 (rows of several coefficients, which do not fit in registers) every
// tile is.
template <typename CT, int LP, int KR>
__device__ __forceinline__ void rx_merge_body(const RxArgs& A, const GateTrig& g) {
    constexpr bool kStageC = LP * sizeof(CT) <= 8;  // coefficients staged in LDS (and held in registers)
    static_assert(KR == 0 || kStageC, "only rows staged in LDS are held in registers");
    constexpr int KH = KR > 0 ? KR : 1;             // size of the hold arrays
    // wider rows are read and written in 16-byte chunks, one thread per chunk
    // (coalesced; a thread always takes the same chunk of a row, so it keeps
    // the maxima of kVPC lanes only)
    constexpr int kCPR = kStageC ? 1 : int(LP * sizeof(CT)) / 16;  // chunks per row
    constexpr int kVPC = kStageC ? LP : LP / kCPR;                  // lanes per chunk
    static_assert(kStageC || (kCPR >= 1 && 64 % kCPR == 0 && kVPC * kCPR == LP), "row chunks");
    __shared__ ulonglong2 sX[kRxTileMax];
    __shared__ ulonglong2 sZ[kRxTileMax];
    __shared__ CT sC[kStageC ? kRxTileMax * LP : 1];
    __shared__ uint16_t sStart[kRxTileMax + 2];
    __shared__ uint16_t sMidx[kRxTileMax];
    __shared__ uint8_t sAlive[kRxTileMax];
    __shared__ uint32_t sOut[2][kRxTileMax];
    __shared__ uint32_t sWave[4];
    __shared__ uint32_t sTile;
    __shared__ uint64_t sBase[2];
    __shared__ TileDesc sDesc[2];  // boundaries of the current tile
    __shared__ double sThr[LP];

    Ctrl* ctrl = A.ctrl;
    const CT* __restrict__ Cin = static_cast<const CT*>(A.Cin);
    CT* __restrict__ Cout = static_cast<CT*>(A.Cout);
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const bool skip = ctrl->err != 0u;
    const uint64_t nf = ctrl->nf[A.in_buf];
    const uint64_t n = nf + ctrl->nb[A.in_buf];
    const uint64_t ntiles = skip ? 0 : (n + kRxTile - 1) / kRxTile;
    const uint32_t ep = ctrl->epoch;
    const bool filt = A.eps_in > 0.0;
    if (tid < LP) sThr[tid] = filt ? A.eps_in * bits_to_d(ctrl->maxbits[A.mx_in][tid]) : -1.0;
    double vmax[kVPC];  // staged rows: every lane; wider rows: the lanes of this thread's chunk
#pragma unroll
    for (int a = 0; a < kVPC; ++a) vmax[a] = 0.0;
    const int zw = g.zword;
    const uint64_t zmask = 1ull << g.zbit;
    const uint64_t cap = A.cap;
    // look-back channels: wave 0 the front run, wave 1 the back run
    const uint64_t gmax = A.max_tiles / 64 + 2;
    uint64_t* const st = A.status + (wave & 1) * A.max_tiles;
    uint64_t* const gst = A.status + 2 * A.max_tiles + (wave & 1) * gmax;

    // the held tile: planned, counts published, outputs in registers
    uint32_t h_tile = kNoTile, h_totA = 0, h_totB = 0;
    uint64_t hxl[KH], hxh[KH], hzl[KH], hzh[KH];  // (scalar words: kept in registers)
    CT hc[KH][kStageC ? LP : 1];

    // ---- this gate's tile boundaries, shared out over the grid's waves
    TileDescWords* const desc = reinterpret_cast<TileDescWords*>(A.desc);
    if (!skip && !A.no_prologue) rx_boundaries(VIn{A.Xin, A.Zin, nf, cap}, n, desc, ep);

    // Each iteration loads and plans a tile (while there are tiles), writes
    // the tile held from the iteration before and holds the new one.  A tile
    // is taken only when the workgroup is about to load it: a tile taken
    // earlier (e.g. while the held tile's offsets resolve) sits unpublished
    // behind that wait, and every later tile's look-back waits for it.
    uint32_t tile = acquire_tile(ctrl, &sTile);
    for (;;) {
        const bool have = tile < ntiles;
        if (!have && h_tile == kNoTile) break;
        RxTile T{};
        uint32_t totA = 0, totB = 0;
        if (have) {
            rx_read_boundaries(VIn{A.Xin, A.Zin, nf, cap}, n, desc, tile, ep, sDesc, &sWave[0]);
            T = rx_tile(sDesc[0], sDesc[1], n);
            if (!T.sane && tid == 0) atomicOr(&ctrl->err, kErrInternal);
            const uint32_t m = T.m;

            // ---- keys (and coefficients) of the tile into LDS.  Every slot loads
            // (slots past the tile end re-read string 0 of the tile), so the values
            // stay in registers and all loads are in flight together.
            if (m > 0) {
                uint64_t rxl[kRxIPT], rxh[kRxIPT], rzl[kRxIPT], rzh[kRxIPT];
                CT rc[kRxIPT][kStageC ? LP : 1];
#pragma unroll
                for (int k = 0; k < kRxIPT; ++k) {
                    const uint32_t e = k * kThreads + tid;
                    const uint64_t p = rx_phys(T, e < m ? e : 0u, nf, cap);
                    const ulonglong2 x = A.Xin[p], z = A.Zin[p];
                    rxl[k] = x.x;
                    rxh[k] = x.y;
                    rzl[k] = z.x;
                    rzh[k] = z.y;
                    if constexpr (kStageC) {
#pragma unroll
                        for (int a = 0; a < LP; ++a) rc[k][a] = Cin[p * LP + a];
                    }
                }
#pragma unroll
                for (int k = 0; k < kRxIPT; ++k) {
                    const uint32_t e = k * kThreads + tid;
                    if (e < m) {
                        sX[e] = make_ulonglong2(rxl[k], rxh[k]);
                        sZ[e] = make_ulonglong2(rzl[k], rzh[k]);
                        if constexpr (kStageC) {
                            bool keep = !filt;
#pragma unroll
                            for (int a = 0; a < LP; ++a) {
                                sC[e * LP + a] = rc[k][a];
                                keep |= absd(rc[k][a]) > sThr[a];
                            }
                            sAlive[e] = uint8_t(keep);
                        } else if (!filt) {
                            sAlive[e] = 1;
                        }
                    }
                }
                if constexpr (!kStageC) {
                    if (filt) {  // a row is alive when some lane is above its threshold: chunks, then OR
                        // kRxBatch chunks per thread at a time (loads in flight together)
                        const uint32_t nc = (m * kCPR + kThreads * kRxBatch - 1) / (kThreads * kRxBatch) *
                                            (kThreads * kRxBatch);
                        for (uint32_t c0 = tid; c0 < nc; c0 += kThreads * kRxBatch) {
                            CT va[kRxBatch][kVPC];
#pragma unroll
                            for (int u = 0; u < kRxBatch; ++u) {
                                const uint32_t c = c0 + uint32_t(u) * kThreads, e = c / kCPR, q = c % kCPR;
                                if (e < m) {
                                    const CT* src = Cin + rx_phys(T, e, nf, cap) * LP + q * kVPC;
#pragma unroll
                                    for (int j = 0; j < kVPC; ++j) va[u][j] = src[j];
                                }
                            }
#pragma unroll
                            for (int u = 0; u < kRxBatch; ++u) {
                                const uint32_t c = c0 + uint32_t(u) * kThreads, e = c / kCPR, q = c % kCPR;
                                int keep = 0;
                                if (e < m) {
#pragma unroll
                                    for (int j = 0; j < kVPC; ++j) keep |= absd(va[u][j]) > sThr[q * kVPC + j];
                                }
#pragma unroll
                                for (int o = 1; o < kCPR; o <<= 1) keep |= __shfl_xor(keep, o, 64);
                                if (e < m && q == 0) sAlive[e] = uint8_t(keep);
                            }
                        }
                    }
                }
            }
            __syncthreads();

            // ---- x-groups ("parts"): ids and starts (blocked: thread owns e0..e0+IPT-1)
            const uint32_t e0 = tid * kRxIPT;
            uint32_t flags = 0, cnt = 0;
#pragma unroll
            for (int k = 0; k < kRxIPT; ++k) {
                const uint32_t e = e0 + k;
                const bool f = e < m && (e == 0 || !k_eq(sX[e], sX[e - 1]));
                flags |= uint32_t(f) << k;
                cnt += f;
            }
            uint32_t npart;
            uint32_t pid = block_excl_scan(cnt, sWave, npart);
            const uint32_t pid0 = pid;
#pragma unroll
            for (int k = 0; k < kRxIPT; ++k) {
                if ((flags >> k) & 1u) sStart[pid++] = uint16_t(e0 + k);
            }
            if (tid == 0) {
                sStart[npart] = uint16_t(m);
                sStart[npart + 1] = uint16_t(m);
            }
            __syncthreads();

            // ---- merged position of every string (merge by z of the two x-groups of a block)
            {
                uint32_t p = pid0;
#pragma unroll
                for (int k = 0; k < kRxIPT; ++k) {
                    const uint32_t e = e0 + k;
                    if (e >= m) continue;
                    if ((flags >> k) & 1u) ++p;
                    const uint32_t mypart = p - 1;
                    const ulonglong2 xe = sX[e], ze = sZ[e];
                    uint32_t os = 0, oe = 0, mpos;
                    if ((xe.x & 1ull) == 0) {
                        if (mypart + 1 < npart) {
                            const uint32_t s = sStart[mypart + 1];
                            if (sX[s].x == (xe.x | 1ull) && sX[s].y == xe.y) {
                                os = s;
                                oe = sStart[mypart + 2];
                            }
                        }
                        uint32_t lo = os, hi = oe;  // partner-group strings with z < ze
                        while (lo < hi) {
                            const uint32_t mid = (lo + hi) >> 1;
                            if (k_lt(sZ[mid], ze)) lo = mid + 1;
                            else hi = mid;
                        }
                        mpos = e + (lo - os);
                    } else {
                        const uint32_t ps = sStart[mypart];
                        if (mypart >= 1) {
                            const uint32_t s = sStart[mypart - 1];
                            if (sX[s].x == (xe.x & ~1ull) && sX[s].y == xe.y) {
                                os = s;
                                oe = ps;
                            }
                        }
                        uint32_t lo = os, hi = oe;  // partner-group strings with z <= ze
                        while (lo < hi) {
                            const uint32_t mid = (lo + hi) >> 1;
                            if (k_le(sZ[mid], ze)) lo = mid + 1;
                            else hi = mid;
                        }
                        mpos = e - (oe - os) + (lo - os);
                    }
                    if (mpos < m) sMidx[mpos] = uint16_t(e);
                    else atomicOr(&ctrl->err, kErrInternal);
                }
            }
            __syncthreads();

            // ---- emission plan in merged order
            uint32_t entA[kRxIPT], entB[kRxIPT];
            uint32_t cntA = 0, cntB = 0;
#pragma unroll
            for (int k = 0; k < kRxIPT; ++k) {
                entA[k] = entB[k] = 0xFFFFFFFFu;
                const uint32_t q = e0 + k;
                if (q >= m) continue;
                const uint32_t e = sMidx[q];
                if (!sAlive[e]) continue;
                const ulonglong2 xe = sX[e], ze = sZ[e];
                const bool isB = xe.x & 1ull;
                const bool ac = ((zw == 0 ? ze.x : ze.y) & zmask) != 0ull;
                if (!isB) {
                    uint32_t e2 = 0xFFFFu;
                    if (q + 1 < m) {
                        const uint32_t c = sMidx[q + 1];
                        if (sX[c].x == (xe.x | 1ull) && sX[c].y == xe.y && k_eq(sZ[c], ze) && sAlive[c]) e2 = c;
                    }
                    if (e2 != 0xFFFFu) {
                        entA[k] = out_entry(e, e2, ac ? 3u : 0u);
                        entB[k] = out_entry(e2, e, ac ? 3u : 0u);
                    } else if (ac) {
                        if (g.any_c) entA[k] = out_entry(e, 0, 1u);
                        if (g.any_s) entB[k] = out_entry(e, 0, 2u);
                    } else {
                        entA[k] = out_entry(e, 0, 0u);
                    }
                } else {
                    bool paired = false;
                    if (q > 0) {
                        const uint32_t c = sMidx[q - 1];
                        paired = sX[c].x == (xe.x & ~1ull) && sX[c].y == xe.y && k_eq(sZ[c], ze) && sAlive[c];
                    }
                    if (paired) {
                        // emitted by the A string of the pair
                    } else if (ac) {
                        if (g.any_s) entA[k] = out_entry(e, 0, 2u);
                        if (g.any_c) entB[k] = out_entry(e, 0, 1u);
                    } else {
                        entB[k] = out_entry(e, 0, 0u);
                    }
                }
                cntA += entA[k] != 0xFFFFFFFFu;
                cntB += entB[k] != 0xFFFFFFFFu;
            }
            uint32_t totPacked;
            const uint32_t offPacked = block_excl_scan(cntA | (cntB << 16), sWave, totPacked);
            totA = totPacked & 0xFFFFu;
            totB = totPacked >> 16;
            {
                uint32_t oa = offPacked & 0xFFFFu, ob = offPacked >> 16;
#pragma unroll
                for (int k = 0; k < kRxIPT; ++k) {
                    if (entA[k] != 0xFFFFFFFFu) sOut[0][oa++] = entA[k];
                    if (entB[k] != 0xFFFFFFFFu) sOut[1][ob++] = entB[k];
                }
            }

            // ---- publish this tile's output counts
            if (wave < 2) lb2_publish(st, gst, tile, ep, wave ? totB : totA, &ctrl->err);
        }

        // ---- offsets of the held tile (waves 0 and 1)
        if (wave < 2 && h_tile != kNoTile) {
            const uint64_t b = lb2_resolve(st, gst, h_tile, ep, wave ? h_totB : h_totA, &ctrl->err);
            if (lane_id() == 0) sBase[wave] = b;
        }
        __syncthreads();
        // ---- write the held tile at the bases in sBase
        if (h_tile != kNoTile) {
            const uint64_t bA = sBase[0], bB = sBase[1];
            if (h_tile == ntiles - 1 && tid == 0) {
                const uint64_t tf = bA + h_totA, tb = bB + h_totB;
                if (tf + tb > cap) {
                    atomicOr(&ctrl->err, kErrCapacity);
                    atomicMax(reinterpret_cast<unsigned long long*>(&ctrl->need),
                              static_cast<unsigned long long>(tf + tb));
                } else {
                    st_rel(&ctrl->nf[A.out_buf], tf);  // read by the launch's last workgroup
                    st_rel(&ctrl->nb[A.out_buf], tb);
                }
            }
#pragma unroll
            for (int k = 0; k < KR; ++k) {
                const uint32_t j = uint32_t(k) * kThreads + tid;
                if (j >= h_totA + h_totB) continue;
                const bool side = j >= h_totA;
                const uint64_t o = side ? bB + (j - h_totA) : bA + j;
                if (o >= cap) continue;
                const uint64_t po = side ? cap - 1 - o : o;
                A.Xout[po] = make_ulonglong2(hxl[k], hxh[k]);
                A.Zout[po] = make_ulonglong2(hzl[k], hzh[k]);
                CT* dst = Cout + po * LP;
#pragma unroll
                for (int a = 0; a < (kStageC ? LP : 0); ++a) dst[a] = hc[k][a];
            }
        }

        if (!have) {
            h_tile = kNoTile;
        } else if (totA + totB <= uint32_t(KR * kThreads)) {
            // ---- gather this tile's outputs into registers
#pragma unroll
            for (int k = 0; k < KR; ++k) {
                const uint32_t j = uint32_t(k) * kThreads + tid;
                if (j >= totA + totB) continue;
                const bool side = j >= totA;
                const uint32_t en = sOut[side][side ? j - totA : j];
                const uint32_t e = en & 0x3FFu, e2 = (en >> 10) & 0x3FFu, kind = en >> 20;
                const ulonglong2 xe = sX[e], ze = sZ[e];
                const ulonglong2 xo = rotr1_n(make_ulonglong2(side ? (xe.x | 1ull) : (xe.x & ~1ull), xe.y), A.nq);
                hxl[k] = xo.x;
                hxh[k] = xo.y;
                hzl[k] = ze.x;
                hzh[k] = ze.y;
                if constexpr (kStageC) {
#pragma unroll
                    for (int a = 0; a < LP; ++a) {
                        const CT v = rx_value<CT, LP>(g, a, kind, !side, sC[e * LP + a], sC[e2 * LP + a]);
                        hc[k][a] = v;
                        vmax[a] = fmax(vmax[a], absd(v));
                    }
                }
            }
            h_tile = tile;
            h_totA = totA;
            h_totB = totB;
        } else {
            // ---- too many outputs to hold: resolve and write this tile now
            __syncthreads();  // every thread has read sBase
            if (wave < 2) {
                const uint64_t b = lb2_resolve(st, gst, tile, ep, wave ? totB : totA, &ctrl->err);
                if (lane_id() == 0) sBase[wave] = b;
            }
            __syncthreads();
            const uint64_t baseA = sBase[0], baseB = sBase[1];
            if (tile == ntiles - 1 && tid == 0) {
                const uint64_t tf = baseA + totA, tb = baseB + totB;
                if (tf + tb > cap) {
                    atomicOr(&ctrl->err, kErrCapacity);
                    atomicMax(reinterpret_cast<unsigned long long*>(&ctrl->need),
                              static_cast<unsigned long long>(tf + tb));
                } else {
                    st_rel(&ctrl->nf[A.out_buf], tf);  // read by the launch's last workgroup
                    st_rel(&ctrl->nb[A.out_buf], tb);
                }
            }
#pragma unroll 1
            for (int side = 0; side < 2; ++side) {
                const uint32_t tot = side ? totB : totA;
                const uint64_t base = side ? baseB : baseA;
                for (uint32_t i = tid; i < tot; i += kThreads) {
                    const uint32_t en = sOut[side][i];
                    const uint32_t e = en & 0x3FFu, e2 = (en >> 10) & 0x3FFu, kind = en >> 20;
                    const ulonglong2 xe = sX[e];
                    const ulonglong2 xo =
                        rotr1_n(make_ulonglong2(side ? (xe.x | 1ull) : (xe.x & ~1ull), xe.y), A.nq);
                    const uint64_t o = base + i;
                    if (o >= cap) continue;
                    const uint64_t po = side ? cap - 1 - o : o;
                    A.Xout[po] = xo;
                    A.Zout[po] = sZ[e];
                    if constexpr (kStageC) {
                        CT* dst = Cout + po * LP;
                        const CT* ce = sC + e * LP;
                        const CT* ce2 = sC + e2 * LP;
#pragma unroll
                        for (int a = 0; a < LP; ++a) {
                            const CT v = rx_value<CT, LP>(g, a, kind, side == 0, ce[a], ce2[a]);
                            dst[a] = v;
                            vmax[a] = fmax(vmax[a], absd(v));
                        }
                    }
                }
                if constexpr (!kStageC) {  // coefficients in 16-byte chunks, one thread per chunk
                    // kRxBatch chunks per thread at a time: their loads are all in
                    // flight before the first store (one latency per batch)
                    for (uint32_t c0 = tid; c0 < tot * kCPR; c0 += kThreads * kRxBatch) {
                        CT va[kRxBatch][kVPC], vb[kRxBatch][kVPC];
                        uint32_t wk[kRxBatch];  // kind, or 4: nothing to write
                        uint64_t wpo[kRxBatch];
#pragma unroll
                        for (int u = 0; u < kRxBatch; ++u) {
                            const uint32_t c = c0 + uint32_t(u) * kThreads;
                            wk[u] = 4u;
                            wpo[u] = 0;
                            if (c >= tot * kCPR) continue;
                            const uint32_t i = c / kCPR, q = c % kCPR;
                            const uint32_t en = sOut[side][i];
                            const uint32_t e = en & 0x3FFu, e2 = (en >> 10) & 0x3FFu, kind = en >> 20;
                            const uint64_t o = base + i;
                            if (o >= cap) continue;
                            const CT* ce = Cin + rx_phys(T, e, nf, cap) * LP + q * kVPC;
                            const CT* ce2 = Cin + rx_phys(T, kind == 3 ? e2 : e, nf, cap) * LP + q * kVPC;
#pragma unroll
                            for (int j = 0; j < kVPC; ++j) {
                                va[u][j] = ce[j];
                                vb[u][j] = ce2[j];
                            }
                            wk[u] = kind;
                            wpo[u] = (side ? cap - 1 - o : o) * LP + q * kVPC;
                        }
#pragma unroll
                        for (int u = 0; u < kRxBatch; ++u) {
                            if (wk[u] == 4u) continue;
                            const uint32_t q = (c0 + uint32_t(u) * kThreads) % kCPR;
                            CT* dst = Cout + wpo[u];
#pragma unroll
                            for (int j = 0; j < kVPC; ++j) {
                                const CT v = rx_value<CT, LP>(g, int(q) * kVPC + j, wk[u], side == 0, va[u][j], vb[u][j]);
                                dst[j] = v;
                                vmax[j] = fmax(vmax[j], absd(v));
                            }
                        }
                    }
                }
            }
            h_tile = kNoTile;
        }
        // the next tile (acquire_tile's barrier also frees this tile's LDS)
        tile = have ? acquire_tile(ctrl, &sTile) : kNoTile;
    }

    // ---- per-lane max of the outputs (wider rows: lane q kVPC + j is held by
    // the threads whose chunk is q, i.e. lane index q modulo kCPR), over the
    // waves through LDS, then one atomic per lane and workgroup: the
    // workgroups leave within a few microseconds of each other, and atomics
    // on one word from all of them queue behind each other
    __shared__ unsigned long long sWmax[LP];  // bit patterns of non-negative doubles order like the values
    if (tid < LP) sWmax[tid] = 0ull;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kVPC; ++j) {
        double mx = vmax[j];
#pragma unroll
        for (int o = kCPR; o < 64; o <<= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
        const int q = lane_id();
        if (q < kCPR && mx > 0.0) atomicMax(&sWmax[q * kVPC + j], static_cast<unsigned long long>(d_to_bits(mx)));
    }
    __syncthreads();
    if (tid < LP && sWmax[tid] != 0ull)
        atomicMax(reinterpret_cast<unsigned long long*>(&ctrl->maxbits[A.mx_out][tid]), sWmax[tid]);
    if (finish_launch(ctrl)) {
        // a failed stage keeps its input (and the input's max) for the re-run
        if (__hip_atomic_load(&ctrl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
            for (int a = 0; a < kMaxLanes; ++a) ctrl->maxbits[A.mx_in][a] = 0ull;
            uint64_t n_out = 0;
            if (ntiles == 0) {
                ctrl->nf[A.out_buf] = 0;
                ctrl->nb[A.out_buf] = 0;
            } else {
                n_out = ld_acq(&ctrl->nf[A.out_buf]) + ld_acq(&ctrl->nb[A.out_buf]);
            }
            ctrl->stages_done += 1;
            ctrl->cnt_updates += n;
            ctrl->cnt_rx_in += n;
            ctrl->cnt_rx_out += n_out;
            ctrl->cnt_rx_launches += 1;
        }
    }
}

// Rows of one coefficient (or two binary32 lanes): outputs held in registers,
// four workgroups per CU (LDS allows four; the register budget is held to it).
template <typename CT, int LP>
__global__ __launch_bounds__(kThreads, 4) void k_rx_merge(RxArgs A, GateTrig g) {
    rx_merge_body<CT, LP, kRxHold>(A, g);
}

// Wider rows: every tile written as soon as its offsets are known.
template <typename CT, int LP>
__global__ __launch_bounds__(kThreads, 4) void k_rx_merge_wide(RxArgs A, GateTrig g) {
    rx_merge_body<CT, LP, 0>(A, g);
}

// ================================================================ Clifford pass / compaction
// Reads the virtual input array, applies the pending truncation, then (if the
// run has generators) a run of Z-only Clifford rotations, and writes the
// survivors compacted to the front of the output.  rank_out (optional)
// receives the index of each string's x-group, the major key of the re-sort.
//
// One Z-only generator J at a Clifford angle maps an anticommuting string
// sigma_I (Eq. update_rule with cos = 0 or sin = 0) to sin(theta) i sigma_J
// sigma_I = sin(theta) (-1)^[e = 1 mod 4] sigma_K, K = (x, z ^ z_J), with
// e = |x & z_K| - |x & z_I|, or to cos(theta) sigma_I.  The generators of a
// run commute, so their product is applied at once: z_f = z ^ (XOR of z_J
// over the anticommuting generators with sin = +-1), and the product of the
// factors (-1)^[e_k = 1 mod 4] = i^(e_k + 1) telescopes to
// i^(|x & z_f| - |x & z| + K), K the number of those generators; the
// negative sin or cos of each anticommuting generator adds its own sign.

__device__ __forceinline__ ulonglong2 shr128(const ulonglong2& v, uint32_t d) {  // 0 < d < 128
    if (d >= 64u) return make_ulonglong2(v.y >> (d - 64u), 0ull);
    return make_ulonglong2((v.x >> d) | (v.y << (64u - d)), v.y >> d);
}

__device__ __forceinline__ ulonglong2 shl128(const ulonglong2& v, uint32_t d) {  // 0 < d < 128
    if (d >= 64u) return make_ulonglong2(0ull, v.x << (d - 64u));
    return make_ulonglong2(v.x << d, (v.y << d) | (v.x >> (64u - d)));
}

template <typename CT, int LP>
__global__ __launch_bounds__(kThreads) void k_compact(CompactArgs A) {
    __shared__ CliffGen sG[kMaxCliffGens];
    __shared__ CliffGroup sGrp[kMaxCliffGroups];
    __shared__ uint32_t sWave[4];
    __shared__ uint32_t sTile;
    __shared__ uint64_t sBase[2];
    __shared__ double sThr[LP];
    __shared__ double sThrL[LP];

    Ctrl* ctrl = A.ctrl;
    const CT* __restrict__ Cin = static_cast<const CT*>(A.Cin);
    CT* __restrict__ Cout = static_cast<CT*>(A.Cout);
    const int tid = threadIdx.x, wave = tid >> 6;
    const bool skip = ctrl->err != 0u;
    const uint64_t nf = ctrl->nf[A.in_buf];
    const uint64_t n = A.prefix_only ? ctrl->prefix_len : nf + ctrl->nb[A.in_buf];
    const uint64_t ntiles = skip ? 0 : (n + kCompactTile - 1) / kCompactTile;
    const uint32_t ep = ctrl->epoch;
    const bool filt = A.eps_in > 0.0;
    // learned rule, unless its estimated error exceeds the tolerance in some
    // lane: then this pass applies the magnitude rule alone (the fallback)
    bool use_learned = A.gscore != nullptr;
    if (use_learned && A.learned_tol > 0.0) {
#pragma unroll
        for (int a = 0; a < LP; ++a) use_learned &= !(ctrl->learned_est[a] > A.learned_tol);
    }
    if (tid < LP) {
        const double M = bits_to_d(ctrl->maxbits[A.mx_in][tid]);
        sThr[tid] = filt ? A.eps_in * M : -1.0;
        sThrL[tid] = A.eps_learned * M;
    }
    for (int i = tid; i < A.ngens; i += kThreads) sG[i] = A.gens[i];
    for (int i = tid; i < A.ngroups; i += kThreads) sGrp[i] = A.groups[i];
    const bool cliff = A.ngens > 0 || A.ngroups > 0;
    double vmax[LP];
#pragma unroll
    for (int a = 0; a < LP; ++a) vmax[a] = 0.0;
    __syncthreads();

    for (;;) {
        const uint32_t tile = acquire_tile(ctrl, &sTile);
        if (tile >= ntiles) break;
        // wave-striped: wave w owns 64 * IPT consecutive strings, element k of
        // a lane is string seg + 64 k + lane (coalesced loads and stores);
        // offsets in input order from ballots, wave bases from one block scan
        const uint64_t seg = uint64_t(tile) * kCompactTile + uint64_t(wave) * 64 * kCompactIPT;
        const int lane = lane_id();
        const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        ulonglong2 xs[kCompactIPT], zs[kCompactIPT];
        CT cs[kCompactIPT][LP];
        uint64_t balA[kCompactIPT], balG[kCompactIPT];
#pragma unroll
        for (int k = 0; k < kCompactIPT; ++k) {
            const uint64_t i = seg + uint64_t(k) * 64 + lane;
            bool al = false, gs = false;
            xs[k] = make_ulonglong2(0, 0);
            zs[k] = make_ulonglong2(0, 0);
#pragma unroll
            for (int a = 0; a < LP; ++a) cs[k][a] = CT(0);
            if (i < n) {
                const uint64_t p = vphys(i, nf, A.cap);
                xs[k] = A.Xin[p];
                zs[k] = A.Zin[p];
#pragma unroll
                for (int a = 0; a < LP; ++a) cs[k][a] = Cin[p * LP + a];
                al = true;
                if (filt) al = keep_row<CT, LP>(cs[k], sThr);
                if (use_learned) {  // learned rule: |c| * min(1, 10^y) > eps * M in some lane
                    const double gw = fmin(1.0, exp10(static_cast<double>(A.gscore[i])));
                    bool keepL = false;
#pragma unroll
                    for (int a = 0; a < LP; ++a) keepL |= absd(cs[k][a]) * gw > sThrL[a];
                    al = al && keepL;
                }
            }
            // a group starts where x differs from the string before (the lane
            // before holds it; lane 0 reads it)
            ulonglong2 xp = shfl_u128(xs[k], lane > 0 ? lane - 1 : 0);
            if (lane == 0 && i < n && i > 0) xp = A.Xin[vphys(i - 1, nf, A.cap)];
            if (i < n) gs = (i == 0) || !k_eq(xp, xs[k]);
            balA[k] = __ballot(al);
            balG[k] = __ballot(gs);
        }
        uint32_t nal = 0, ngs = 0;
#pragma unroll
        for (int k = 0; k < kCompactIPT; ++k) {
            nal += uint32_t(__popcll(balA[k]));
            ngs += uint32_t(__popcll(balG[k]));
        }
        uint32_t totPacked;
        const uint32_t wOff = __shfl(block_excl_scan(lane == 0 ? (nal | (ngs << 16)) : 0u, sWave, totPacked), 0);
        // publish this tile's counts first, then apply the run's product to the
        // surviving strings (zs[k] becomes z_f; negs bit k: the product
        // negates it) while the predecessors' prefixes arrive
        if (wave == 0) lookback_publish(A.status, 1, tile, ep, totPacked & 0xFFFFu);
        else if (wave == 1) lookback_publish(A.status + A.max_tiles, 1, tile, ep, totPacked >> 16);
        uint32_t negs = 0;
        if (cliff) {
#pragma unroll
            for (int k = 0; k < kCompactIPT; ++k) {
                if (!((balA[k] >> lane) & 1ull)) continue;
                ulonglong2 z = zs[k];
                bool neg = false;
                {
                    const ulonglong2 x = rotl_n(xs[k], A.xrot, A.nq);
                    int K = 0, nneg = 0;
                    for (int gi = 0; gi < A.ngroups; ++gi) {
                        // bit a of c: x_a != x_(a+d), i.e. Z_a Z_(a+d) anticommutes
                        const uint32_t d = __builtin_amdgcn_readfirstlane(sGrp[gi].d);
                        const ulonglong2 y = shr128(x, d);
                        const uint64_t c0 = x.x ^ y.x, c1 = x.y ^ y.y;
                        const ulonglong2 ck = make_ulonglong2(c0 & sGrp[gi].k0, c1 & sGrp[gi].k1);
                        const ulonglong2 up = shl128(ck, d);
                        z.x ^= ck.x ^ up.x;
                        z.y ^= ck.y ^ up.y;
                        K += __popcll(ck.x) + __popcll(ck.y);
                        if (!A.groups_neg_is_k) nneg += __popcll(c0 & sGrp[gi].n0) + __popcll(c1 & sGrp[gi].n1);
                    }
                    if (A.groups_neg_is_k) nneg = K;  // every grouped generator with sin = -1
                    for (int gi = 0; gi < A.ngens; ++gi) {
                        const CliffGen G = sG[gi];
                        if (!((__popcll(x.x & G.z0) + __popcll(x.y & G.z1)) & 1)) continue;
                        if (G.kodd) {
                            z.x ^= G.z0;
                            z.y ^= G.z1;
                            ++K;
                        }
                        nneg += int(G.neg);
                    }
                    const int e = k_popc_and(x, z) - k_popc_and(x, zs[k]) + K;  // even
                    neg = ((e & 3) == 2) != ((nneg & 1) != 0);
                }
                negs |= uint32_t(neg) << k;
                zs[k] = z;
            }
        }
        if (wave == 0) {
            const uint64_t b = lookback_resolve(A.status, 1, tile, ep, totPacked & 0xFFFFu, &ctrl->err);
            if (lane_id() == 0) sBase[0] = b;
        } else if (wave == 1) {
            const uint64_t b = lookback_resolve(A.status + A.max_tiles, 1, tile, ep, totPacked >> 16, &ctrl->err);
            if (lane_id() == 0) sBase[1] = b;
        }
        __syncthreads();
        uint64_t oW = sBase[0] + (wOff & 0xFFFFu);  // survivors before element k of this wave
        uint64_t rW = sBase[1] + (wOff >> 16);      // group starts before element k of this wave
        if (tile == ntiles - 1 && tid == 0) {
            st_rel(&ctrl->nf[A.out_buf], sBase[0] + (totPacked & 0xFFFFu));  // read by the last workgroup
            st_rel(&ctrl->nb[A.out_buf], 0ull);
            if (!A.prefix_only) st_rel(&ctrl->nranks, sBase[1] + (totPacked >> 16));
        }
#pragma unroll
        for (int k = 0; k < kCompactIPT; ++k) {
            const uint64_t o = oW + uint64_t(__popcll(balA[k] & lt_mask));
            const uint64_t rk = rW + uint64_t(__popcll(balG[k] & lt_mask)) + ((balG[k] >> lane) & 1ull);
            oW += uint64_t(__popcll(balA[k]));
            rW += uint64_t(__popcll(balG[k]));
            if (!((balA[k] >> lane) & 1ull)) continue;
            const bool neg = (negs >> k) & 1u;
            const ulonglong2 z = zs[k];
            A.Xout[o] = xs[k];
            A.Zout[o] = z;
            if (A.rank_out) A.rank_out[o] = uint32_t(rk - 1);
#pragma unroll
            for (int a = 0; a < LP; ++a) {
                const CT v = neg ? -cs[k][a] : cs[k][a];
                Cout[o * LP + a] = v;
                vmax[a] = fmax(vmax[a], absd(v));
            }
        }
        __syncthreads();
    }
    if (!A.prefix_only) {  // over the waves through LDS, then one atomic per lane and workgroup
        __shared__ unsigned long long sWmax[LP];
        if (tid < LP) sWmax[tid] = 0ull;
        __syncthreads();
#pragma unroll
        for (int a = 0; a < LP; ++a) {
            const double mx = wave_max_d(vmax[a]);
            if (lane_id() == 0 && mx > 0.0) atomicMax(&sWmax[a], static_cast<unsigned long long>(d_to_bits(mx)));
        }
        __syncthreads();
        if (tid < LP && sWmax[tid] != 0ull)
            atomicMax(reinterpret_cast<unsigned long long*>(&ctrl->maxbits[A.mx_out][tid]), sWmax[tid]);
    }
    if (finish_launch(ctrl)) {
        if (A.prefix_only) {
            if (ntiles == 0) {
                ctrl->nf[A.out_buf] = 0;
                ctrl->nb[A.out_buf] = 0;
            }
            ctrl->prefix_len = __hip_atomic_load(&ctrl->nf[A.out_buf], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (__hip_atomic_load(&ctrl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
            for (int a = 0; a < kMaxLanes; ++a) ctrl->maxbits[A.mx_in][a] = 0ull;
            if (ntiles == 0) {
                ctrl->nf[A.out_buf] = 0;
                ctrl->nb[A.out_buf] = 0;
                ctrl->nranks = 0;
            }
            ctrl->stages_done += 1;
            ctrl->cnt_updates += n * uint64_t(A.gate_count);
            ctrl->cnt_cliff_in += n;
            ctrl->cnt_cliff_launches += 1;
            if (A.gscore) {
                ctrl->learned_passes += 1;
                if (!use_learned) ctrl->learned_fallbacks += 1;
            }
        }
    }
}

// ================================================================ onesweep radix sort
// LSD radix sort, one stable pass per digit, with decoupled look-back across
// tiles for the bucket offsets (Adinets & Merrill, "Onesweep", 2022).  The
// digit width (1..8 bits) and the tile size are chosen per sort by the host.

// Bits [lo, lo + w) of the key integer whose 64-bit words, least significant
// first, are z.x, z.y, r, x.x, x.y.  A digit may straddle two words.
__device__ __forceinline__ uint64_t key_word(int i, uint32_t r, const ulonglong2& z, const ulonglong2& x) {
    return i == 0 ? z.x : i == 1 ? z.y : i == 2 ? uint64_t(r) : i == 3 ? x.x : x.y;
}

__device__ __forceinline__ uint32_t key_digit(int lo, int w, uint32_t r, const ulonglong2& z, const ulonglong2& x) {
    const int i = lo >> 6, sh = lo & 63;
    uint64_t v = key_word(i, r, z, x) >> sh;
    if (sh + w > 64) v |= key_word(i + 1, r, z, x) << (64 - sh);
    return uint32_t(v) & ((1u << w) - 1u);
}

__global__ __launch_bounds__(kThreads) void k_sort_hist(const Ctrl* __restrict__ ctrl, int buf,
                                                        const uint32_t* __restrict__ R,
                                                        const ulonglong2* __restrict__ Z,
                                                        const ulonglong2* __restrict__ X, SortPlan plan,
                                                        uint32_t* __restrict__ hist) {
    __shared__ uint32_t sh[kSortMaxPasses][256];
    const int np = plan.npass;
    const bool need_x = np > 0 && plan.lo[np - 1] + plan.w[np - 1] > 192;  // passes ascend in lo
    const bool need_z = np > 0 && plan.lo[0] < 128;
    for (int i = threadIdx.x; i < np * 256; i += kThreads) (&sh[0][0])[i] = 0;
    __syncthreads();
    const uint64_t n = ctrl->nf[buf];
    if (!ctrl->err) {
        for (uint64_t i = blockIdx.x * uint64_t(kThreads) + threadIdx.x; i < n; i += uint64_t(gridDim.x) * kThreads) {
            const ulonglong2 z = need_z ? Z[i] : ulonglong2{0, 0};
            const ulonglong2 x = need_x ? X[i] : ulonglong2{0, 0};
            const uint32_t r = R ? R[i] : 0u;
            for (int p = 0; p < np; ++p) atomicAdd(&sh[p][key_digit(plan.lo[p], plan.w[p], r, z, x)], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < np * 256; i += kThreads) {
        const uint32_t v = (&sh[0][0])[i];
        if (v) atomicAdd(hist + i, v);
    }
}

template <typename CT, int LP, int IPT>
__global__ __launch_bounds__(kThreads) void k_sort_pass(SortPassArgs A) {
    constexpr int kTile = kThreads * IPT;
    __shared__ uint32_t sCnt[4][256];
    __shared__ uint64_t sOff[4][256];
    __shared__ uint32_t sTile;
    Ctrl* ctrl = A.ctrl;
    const CT* __restrict__ Cs = static_cast<const CT*>(A.Cs);
    CT* __restrict__ Cd = static_cast<CT*>(A.Cd);
    const int tid = threadIdx.x, wave = tid >> 6, lane = lane_id();
    const bool skip = ctrl->err != 0u;
    const uint64_t ntiles = skip ? 0 : (A.n + kTile - 1) / kTile;
    const uint32_t ep = ctrl->epoch;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int w = A.w, nbk = 1 << A.w;
    const bool has_r = A.Rs != nullptr;

    for (;;) {
        const uint32_t tile = acquire_tile(ctrl, &sTile);
        if (tile >= ntiles) break;
        for (int i = tid; i < 4 * 256; i += kThreads) (&sCnt[0][0])[i] = 0;
        __syncthreads();
        // warp-striped: wave w owns a contiguous segment of 64*IPT strings
        const uint64_t seg = uint64_t(tile) * kTile + uint64_t(wave) * 64 * IPT;
        uint32_t dig[IPT];
        uint32_t loc[IPT];
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            const uint64_t i = seg + uint64_t(k) * 64 + lane;
            const bool valid = i < A.n;
            uint32_t d = 0;
            if (valid) d = key_digit(A.lo, w, has_r ? A.Rs[i] : 0u, A.Zs[i], A.Xs[i]);
            dig[k] = valid ? d : 0xFFFFFFFFu;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                if (b < w) {
                    const uint64_t bb = __ballot((d >> b) & 1u);
                    peers &= ((d >> b) & 1u) ? bb : ~bb;
                }
            }
            uint32_t pre = 0;
            if (valid) pre = sCnt[wave][d];
            const uint32_t below = __popcll(peers & lt_mask);
            loc[k] = pre + below;
            if (valid && below == 0) sCnt[wave][d] = pre + __popcll(peers);
        }
        __syncthreads();
        // per bucket: prefix over waves, tile total, look-back across tiles
        if (tid < nbk) {
            const int d = tid;
            const uint32_t c0 = sCnt[0][d], c1 = sCnt[1][d], c2 = sCnt[2][d], c3 = sCnt[3][d];
            const uint32_t tot = c0 + c1 + c2 + c3;
            const uint64_t excl = lookback_thread(A.status + d, 256, tile, ep, tot, &ctrl->err);
            const uint64_t b = uint64_t(A.digit_base[d]) + excl;
            sOff[0][d] = b;
            sOff[1][d] = b + c0;
            sOff[2][d] = b + c0 + c1;
            sOff[3][d] = b + c0 + c1 + c2;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < IPT; ++k) {
            if (dig[k] == 0xFFFFFFFFu) continue;
            const uint64_t i = seg + uint64_t(k) * 64 + lane;
            const uint64_t o = sOff[wave][dig[k]] + loc[k];
            if (o >= A.n) continue;  // cannot happen for a consistent histogram
            if (has_r) A.Rd[o] = A.Rs[i];
            A.Zd[o] = A.Zs[i];
            A.Xd[o] = A.Xs[i];
#pragma unroll
            for (int a = 0; a < LP; ++a) Cd[o * LP + a] = Cs[i * LP + a];
            if (A.Ls) {
#pragma unroll
                for (int a = 0; a < LP; ++a) A.Ld[o * LP + a] = A.Ls[i * LP + a];
            }
        }
        __syncthreads();
    }
    if (finish_launch(ctrl)) {
        if (!skip) {
            ctrl->nf[A.dst_buf] = A.n;
            ctrl->nb[A.dst_buf] = 0;
        }
    }
}

// ================================================================ reductions
// mode 0: <Z> = sum of c over the x == 0 prefix; mode 1: sum of c^2 over all.
// Deterministic: fixed chunk per block, fixed tree, fixed final order.

__global__ void k_prefix_len(Ctrl* ctrl, int buf, const ulonglong2* __restrict__ X, uint64_t cap) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint64_t nf = ctrl->nf[buf];
    uint64_t lo = 0, hi = nf;  // x == 0 strings precede all others and sit in the front run
    while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        const ulonglong2 x = X[mid];
        if (x.x == 0 && x.y == 0) lo = mid + 1;
        else hi = mid;
    }
    ctrl->prefix_len = lo;
}

// eps_pend > 0 (mode 1 only): strings the pending truncation drops (|c| <=
// eps_pend * max |c| in every lane, max from slot mx) contribute nothing.
template <typename CT, int LP>
__global__ __launch_bounds__(kThreads) void k_reduce_partial(const Ctrl* __restrict__ ctrl, int buf,
                                                             const CT* __restrict__ C, uint64_t cap, int mode,
                                                             double eps_pend, int mx,
                                                             double* __restrict__ partial) {
    __shared__ double sAcc[4][LP];
    __shared__ double sThr[LP];
    const bool filt = mode == 1 && eps_pend > 0.0;
    if (threadIdx.x < LP) sThr[threadIdx.x] = filt ? eps_pend * bits_to_d(ctrl->maxbits[mx][threadIdx.x]) : -1.0;
    __syncthreads();
    const uint64_t nf = ctrl->nf[buf];
    const uint64_t len = (mode == 0) ? ctrl->prefix_len : nf + ctrl->nb[buf];
    const uint64_t chunk = (len + gridDim.x - 1) / gridDim.x;
    const uint64_t b0 = blockIdx.x * chunk;
    const uint64_t b1 = (b0 + chunk < len) ? b0 + chunk : len;
    double acc[LP];
#pragma unroll
    for (int a = 0; a < LP; ++a) acc[a] = 0.0;
    for (uint64_t i = b0 + threadIdx.x; i < b1; i += kThreads) {
        const uint64_t p = vphys(i, nf, cap);
        if (filt && !keep_row<CT, LP>(C + p * LP, sThr)) continue;
#pragma unroll
        for (int a = 0; a < LP; ++a) {
            const double v = static_cast<double>(C[p * LP + a]);
            acc[a] += (mode == 0) ? v : v * v;
        }
    }
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < LP; ++a) {
        double v = acc[a];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane_id() == 0) sAcc[wave][a] = v;
    }
    __syncthreads();
    if (threadIdx.x < LP) {
        const int a = threadIdx.x;
        partial[blockIdx.x * LP + a] = ((sAcc[0][a] + sAcc[1][a]) + sAcc[2][a]) + sAcc[3][a];
    }
}

// Learned-rule error estimate (deterministic: fixed chunks, fixed trees).
// A string the magnitude rule keeps and the learned rule drops adds
// (|c_a| w)^2 and |c_a| w, w = min(1, 10^y), to lane a.
template <typename CT, int LP>
__global__ __launch_bounds__(kThreads) void k_learned_partial(const Ctrl* __restrict__ ctrl, int buf,
                                                              const CT* __restrict__ C,
                                                              const float* __restrict__ gscore, uint64_t cap,
                                                              double eps_pend, double eps_learned, int mx,
                                                              double* __restrict__ partial) {
    __shared__ double sAcc[4][2][LP];
    __shared__ double sThr[LP], sThrL[LP];
    if (threadIdx.x < LP) {
        const double M = bits_to_d(ctrl->maxbits[mx][threadIdx.x]);
        sThr[threadIdx.x] = eps_pend > 0.0 ? eps_pend * M : -1.0;
        sThrL[threadIdx.x] = eps_learned * M;
    }
    __syncthreads();
    const uint64_t nf = ctrl->nf[buf];
    const uint64_t len = nf + ctrl->nb[buf];
    const uint64_t chunk = (len + gridDim.x - 1) / gridDim.x;
    const uint64_t b0 = blockIdx.x * chunk;
    const uint64_t b1 = (b0 + chunk < len) ? b0 + chunk : len;
    double sq[LP], ab[LP];
#pragma unroll
    for (int a = 0; a < LP; ++a) sq[a] = ab[a] = 0.0;
    for (uint64_t i = b0 + threadIdx.x; i < b1; i += kThreads) {
        const uint64_t p = vphys(i, nf, cap);
        const double w = fmin(1.0, exp10(static_cast<double>(gscore[i])));
        bool keepM = false, keepL = false;
#pragma unroll
        for (int a = 0; a < LP; ++a) {
            const double c = absd(C[p * LP + a]);
            keepM |= c > sThr[a];
            keepL |= c * w > sThrL[a];
        }
        if (!keepM || keepL) continue;
#pragma unroll
        for (int a = 0; a < LP; ++a) {
            const double v = absd(C[p * LP + a]) * w;
            sq[a] += v * v;
            ab[a] += v;
        }
    }
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int a = 0; a < LP; ++a) {
        double u = sq[a], v = ab[a];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            u += __shfl_xor(u, o, 64);
            v += __shfl_xor(v, o, 64);
        }
        if (lane_id() == 0) {
            sAcc[wave][0][a] = u;
            sAcc[wave][1][a] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < 2 * LP) {
        const int q = threadIdx.x / LP, a = threadIdx.x % LP;
        partial[(blockIdx.x * 2 + q) * LP + a] = ((sAcc[0][q][a] + sAcc[1][q][a]) + sAcc[2][q][a]) + sAcc[3][q][a];
    }
}

template <int LP>
__global__ void k_learned_final(const double* __restrict__ partial, int nblocks, Ctrl* ctrl) {
    if (threadIdx.x < 2 * LP) {
        const int q = threadIdx.x / LP, a = threadIdx.x % LP;
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += partial[(b * 2 + q) * LP + a];
        if (q == 0) ctrl->learned_est[a] = sqrt(s);
        else ctrl->learned_l1[a] = s;
    }
}

template <int LP>
__global__ void k_reduce_final(const double* __restrict__ partial, int nblocks, double* __restrict__ out) {
    if (threadIdx.x < LP) {
        const int a = threadIdx.x;
        double s = 0.0;
        for (int b = 0; b < nblocks; ++b) s += partial[b * LP + a];
        out[a] = s;
    }
}

__global__ void k_fill_u64(uint64_t* p, uint64_t v, size_t n) {
    for (size_t i = blockIdx.x * size_t(blockDim.x) + threadIdx.x; i < n; i += size_t(gridDim.x) * blockDim.x)
        p[i] = v;
}

// ================================================================ launchers

// Workgroups of the RX merge for (dtype, padded lanes) one CU holds at once.
int rx_blocks_per_cu(int dtype, int lp) {
    int nb = 0;
    hipError_t e = hipSuccess;
    if (lp * (dtype == 0 ? 8 : 4) <= 8) {
        if (dtype == 0) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rx_merge<double, 1>, kThreads, 0);
        else if (lp == 1) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rx_merge<float, 1>, kThreads, 0);
        else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rx_merge<float, 2>, kThreads, 0);
    } else {
#define O_RX(T, L) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_rx_merge_wide<T, L>, kThreads, 0)
        switch (lp) {
            case 2: if (dtype == 0) O_RX(double, 2); break;
            case 4: if (dtype == 0) O_RX(double, 4); else O_RX(float, 4); break;
            case 8: if (dtype == 0) O_RX(double, 8); else O_RX(float, 8); break;
            case 16: if (dtype == 0) O_RX(double, 16); else O_RX(float, 16); break;
            case 32: if (dtype == 0) O_RX(double, 32); else O_RX(float, 32); break;
            default: break;
        }
#undef O_RX
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb;
}

hipError_t launch_rx(const RxArgs& a, const GateTrig& g, int dtype, int lp, hipStream_t s, int grid) {
    if (lp * (dtype == 0 ? 8 : 4) <= 8) {
        if (dtype == 0) k_rx_merge<double, 1><<<dim3(grid), dim3(kThreads), 0, s>>>(a, g);
        else if (lp == 1) k_rx_merge<float, 1><<<dim3(grid), dim3(kThreads), 0, s>>>(a, g);
        else k_rx_merge<float, 2><<<dim3(grid), dim3(kThreads), 0, s>>>(a, g);
        return hipGetLastError();
    }
#define L_RX(T, L) k_rx_merge_wide<T, L><<<dim3(grid), dim3(kThreads), 0, s>>>(a, g)
    ORQA_DISPATCH(dtype, lp, L_RX);
#undef L_RX
    return hipGetLastError();
}

hipError_t launch_compact(const CompactArgs& a, int dtype, int lp, hipStream_t s, int grid) {
#define L_CP(T, L) k_compact<T, L><<<dim3(grid), dim3(kThreads), 0, s>>>(a)
    ORQA_DISPATCH(dtype, lp, L_CP);
#undef L_CP
    return hipGetLastError();
}

hipError_t launch_sort_hist(Ctrl* ctrl, int buf, const uint32_t* R, const ulonglong2* Z, const ulonglong2* X,
                            const SortPlan& plan, uint32_t* hist, hipStream_t s, int grid) {
    k_sort_hist<<<dim3(grid), dim3(kThreads), 0, s>>>(ctrl, buf, R, Z, X, plan, hist);
    return hipGetLastError();
}

// ================================================================ group sort
// After the Clifford layer the operator is still ordered by x-group; only the
// z order inside each group is lost (every z of a group was XORed with the
// same mask).  The same holds after a general rotation with x_J = 0, whose
// children stay in their parent's group.  When no group exceeds kGsMaxGroup
// strings, each group is sorted by z inside one workgroup, in place of the
// group's positions, so no prefix sum across workgroups is needed.  Workgroup
// tiles cover kGsTile positions and own the groups that start there.  A group
// that would not fit sets ctrl->aux[2] and the caller falls back to the radix
// sort (the input is left untouched).

// The groups a tile owns: [a, b) from the first group start at or after t0 to
// the first at or after t1 (or n): wave 0 looks from t0 and wave 1 from t1,
// 64 positions per step (a string's predecessor from the lane before it).
// Returns 0 when no group starts in the tile, -1 when a group is longer than
// kGsMaxGroup (ctrl->aux[2] is set), 1 otherwise.  Called by the whole
// workgroup.
__device__ int gs_tile_groups(const GroupSortArgs& A, uint64_t n, uint64_t t0, uint64_t t1, uint32_t& sA,
                              uint32_t& sB, uint64_t& a, uint64_t& b) {
    const int wave = threadIdx.x >> 6, lane = lane_id();
    if (wave < 2) {
        const uint64_t base = wave == 0 ? t0 : t1;
        uint32_t found = 0xFFFFFFFFu;
        for (uint32_t c = 0; base < n && c < uint32_t(kGsMaxGroup); c += 64) {
            const uint64_t p = base + c + uint64_t(lane);
            const bool in = p < n;
            const ulonglong2 x = in ? A.Xs[p] : make_ulonglong2(0, 0);
            ulonglong2 prev = shfl_u128(x, lane > 0 ? lane - 1 : 0);
            if (lane == 0 && in && p > 0) prev = A.Xs[p - 1];
            const uint64_t st = __ballot(in && (p == 0 || !k_eq(x, prev)));
            if (st) {
                found = c + uint32_t(__ffsll(static_cast<unsigned long long>(st)) - 1);
                break;
            }
            if (base + c + 64 >= n) break;
        }
        if (lane == 0) {
            if (wave == 0) sA = found;
            else sB = found;
        }
    }
    __syncthreads();
    // A search window of full length without a group start means a group
    // longer than kGsMaxGroup; one cut short by the end of the operator only
    // means that no group starts there.
    const bool full_a = t0 + kGsMaxGroup <= n, full_b = t1 + kGsMaxGroup <= n;
    const bool over = (sA == 0xFFFFFFFFu && full_a) || (t1 < n && sB == 0xFFFFFFFFu && full_b);
    a = sA == 0xFFFFFFFFu ? n : t0 + sA;
    b = (t1 < n && sB != 0xFFFFFFFFu) ? t1 + sB : n;
    __syncthreads();  // sA, sB read by every thread before the next tile sets them
    if (over) {
        if (threadIdx.x == 0) atomicOr(reinterpret_cast<unsigned int*>(&A.ctrl->aux[2]), 1u);
        return -1;
    }
    return a < t1 ? 1 : 0;  // else the tile's strings belong to an earlier tile's group
}

// Any group order: a string's new position is its group's start plus the
// number of group members with a smaller z, equal z counting for the members
// before it (a stable order, so the duplicate keys a rotation creates land
// next to each other).
template <typename CT, int LP>
__global__ __launch_bounds__(kGsThreads) void k_group_sort(GroupSortArgs A) {
    __shared__ ulonglong2 sZ[kGsCap];
    __shared__ uint8_t sF[kGsCap + 1];  // group-start flags, sF[m] = 1 as a sentinel
    __shared__ uint32_t sA, sB;
    Ctrl* ctrl = A.ctrl;
    const CT* __restrict__ Cs = static_cast<const CT*>(A.Cs);
    CT* __restrict__ Cd = static_cast<CT*>(A.Cd);
    const int tid = threadIdx.x;
    const uint64_t n = ctrl->nf[A.in_buf];
    const uint64_t ntiles = ctrl->err ? 0 : (n + kGsTile - 1) / kGsTile;
    if (blockIdx.x == 0 && tid == 0 && ctrl->err == 0u) {
        ctrl->nf[A.out_buf] = n;
        ctrl->nb[A.out_buf] = 0;
    }
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint64_t t0 = tile * kGsTile;
        const uint64_t t1 = t0 + kGsTile < n ? t0 + kGsTile : n;
        uint64_t a, b;
        if (gs_tile_groups(A, n, t0, t1, sA, sB, a, b) <= 0) continue;
        const uint32_t m = uint32_t(b - a);  // <= kGsCap by construction
        // stage z and the group-start flags; keep x and coefficients in registers
        constexpr bool kRegC = LP * sizeof(CT) <= 16;  // wider rows are copied at write time
        ulonglong2 xr[kGsIPT], zr[kGsIPT];
        CT cr[kGsIPT][kRegC ? LP : 1];
#pragma unroll
        for (int k = 0; k < kGsIPT; ++k) {
            const uint32_t e = k * kGsThreads + tid;
            const uint64_t p = a + (e < m ? e : 0u);
            xr[k] = A.Xs[p];
            zr[k] = A.Zs[p];
            if constexpr (kRegC) {
#pragma unroll
                for (int l = 0; l < LP; ++l) cr[k][l] = Cs[p * LP + l];
            }
            if (e < m) {
                sZ[e] = zr[k];
                sF[e] = uint8_t(e == 0 || !k_eq(xr[k], A.Xs[p - 1]));
            }
        }
        if (tid == 0) sF[m] = 1;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kGsIPT; ++k) {
            const uint32_t e = k * kGsThreads + tid;
            if (e >= m) continue;
            const ulonglong2 z = zr[k];
            uint32_t r = 0, j = e;
            while (!sF[j]) {  // members before e in the group (ties count: stable)
                --j;
                r += k_le(sZ[j], z);
            }
            const uint32_t gs = j;
            for (j = e + 1; !sF[j]; ++j) r += k_lt(sZ[j], z);  // members after e
            const uint64_t d = a + gs + r;
            A.Xd[d] = xr[k];
            A.Zd[d] = z;
            if (A.Ls) {
#pragma unroll
                for (int l = 0; l < LP; ++l) A.Ld[d * LP + l] = A.Ls[(a + e) * LP + l];
            }
            if constexpr (kRegC) {
#pragma unroll
                for (int l = 0; l < LP; ++l) Cd[d * LP + l] = cr[k][l];
            } else {
                const uint64_t p = a + e;
#pragma unroll 4
                for (int l = 0; l < LP; ++l) Cd[d * LP + l] = Cs[p * LP + l];
            }
        }
        __syncthreads();
    }
}

// Groups that are z-sorted runs XORed with one mask each (the output of a
// Clifford run, whose input is sorted by (x, z) and whose generators add the
// same z mask to every string of an x-group).  The new order of a group is
// the binary trie of its old keys with the two children of some nodes
// swapped.  The adjacent pair (e-1, e), whose highest differing bit is D_e,
// splits the node [PG, NG) at e, PG the nearest position before e and NG the
// nearest after it whose pair differs in a higher bit (a group start counts as
// higher than any bit); the two halves swap when z_(e-1) > z_e after the XOR,
// which moves [PG, e) right by NG - e and [e, NG) left by e - PG.  The moves
// of all nodes meet in a difference array whose prefix sum is each string's
// displacement inside its group: O(depth of the trie) work per string in
// place of a scan of its whole group.
// High bit of every byte of w (eight entries of D, each <= 126 or 0xFF) that
// is greater than d <= 126: (b | 0x80) - (d + 1) keeps its high bit exactly
// when b & 0x7F > d, and no byte borrows from the next.
__device__ __forceinline__ uint64_t bytes_above(uint64_t w, uint32_t d) {
    constexpr uint64_t kHi = 0x8080808080808080ull, kOne = 0x0101010101010101ull;
    return ((w | kHi) - kOne * uint64_t(d + 1u)) & kHi;
}

__device__ __forceinline__ uint32_t hdb128(const ulonglong2& t) {  // t != 0
    return t.y ? 127u - uint32_t(__clzll(t.y)) : 63u - uint32_t(__clzll(t.x));
}

template <typename CT, int LP>
__global__ __launch_bounds__(kGsThreads, 4) void k_group_sort_xor(GroupSortArgs A) {
    constexpr int kPad = kGsCap + 64;
    constexpr uint8_t kTop = 0xFF;                   // group start, and every entry from m on
    __shared__ __align__(16) uint8_t sD[kPad];        // D_e
    const uint64_t* sW = reinterpret_cast<const uint64_t*>(sD);
    __shared__ uint8_t sBM[kPad / 32];               // maxima of sD over 32-entry blocks
    __shared__ uint32_t sDiff[kGsCap + 1];           // displacements (two's complement)
    __shared__ uint32_t sWave[kGsThreads / 64];
    __shared__ uint32_t sA, sB;
    Ctrl* ctrl = A.ctrl;
    const CT* __restrict__ Cs = static_cast<const CT*>(A.Cs);
    CT* __restrict__ Cd = static_cast<CT*>(A.Cd);
    const int tid = threadIdx.x;
    const uint64_t n = ctrl->nf[A.in_buf];
    const uint64_t ntiles = ctrl->err ? 0 : (n + kGsTile - 1) / kGsTile;
    if (blockIdx.x == 0 && tid == 0 && ctrl->err == 0u) {
        ctrl->nf[A.out_buf] = n;
        ctrl->nb[A.out_buf] = 0;
    }
    for (uint64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const uint64_t t0 = tile * kGsTile;
        const uint64_t t1 = t0 + kGsTile < n ? t0 + kGsTile : n;
        uint64_t a, b;
        if (gs_tile_groups(A, n, t0, t1, sA, sB, a, b) <= 0) continue;
        const uint32_t m = uint32_t(b - a);  // <= kGsCap by construction
        // the coefficients stay in registers until the write; x and z are read
        // again there (the tile's strings are still in the cache).  A string's
        // predecessor is the lane before it (lane 0 reads its own).
        constexpr bool kRegC = LP * sizeof(CT) <= 16;
        CT cr[kGsIPT][kRegC ? LP : 1];
        uint32_t swap = 0;  // bit k: the pair ending at element k swaps its node
        const int lane = lane_id();
        if constexpr (kRegC) {
#pragma unroll
            for (int k = 0; k < kGsIPT; ++k) {
                const uint32_t e = k * kGsThreads + tid;
                const uint64_t p = a + (e < m ? e : 0u);
#pragma unroll
                for (int l = 0; l < LP; ++l) cr[k][l] = Cs[p * LP + l];
            }
        }
#pragma unroll 1
        for (int k = 0; k < kGsIPT; ++k) {
            const uint32_t e = k * kGsThreads + tid;
            if (__ballot(e < m) == 0) break;  // e grows with k
            const uint64_t p = a + (e < m ? e : 0u);
            const ulonglong2 x = A.Xs[p], z = A.Zs[p];
            ulonglong2 xp = shfl_u128(x, lane > 0 ? lane - 1 : 0), zp = shfl_u128(z, lane > 0 ? lane - 1 : 0);
            if (lane == 0 && e != 0 && e < m) {
                xp = A.Xs[p - 1];
                zp = A.Zs[p - 1];
            }
            if (e < m) {
                uint8_t d = kTop;
                if (e != 0 && k_eq(x, xp)) {
                    d = uint8_t(hdb128(make_ulonglong2(zp.x ^ z.x, zp.y ^ z.y)));
                    swap |= uint32_t(k_lt(z, zp)) << k;
                }
                sD[e] = d;
            }
        }
        const uint32_t mend = (m & ~31u) + 64u;  // blocks read by the searches end here
        for (uint32_t i = m + tid; i < mend; i += kGsThreads) sD[i] = kTop;
        for (uint32_t i = tid; i <= m; i += kGsThreads) sDiff[i] = 0u;
        __syncthreads();
        for (uint32_t j = tid; j < mend / 32; j += kGsThreads) {
            const uint32_t* w = reinterpret_cast<const uint32_t*>(sD + 32 * j);
            uint32_t mx = 0;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const uint32_t v = w[q];
                mx = max(mx, max(max(v & 0xFFu, (v >> 8) & 0xFFu), max((v >> 16) & 0xFFu, v >> 24)));
            }
            sBM[j] = uint8_t(mx);
        }
        __syncthreads();
#pragma unroll 1
        for (int k = 0; k < kGsIPT; ++k) {
            if (!((swap >> k) & 1u)) continue;
            const int e = k * kGsThreads + tid;
            const uint8_t d = sD[e];
            // PG: sD[gs] = kTop > d bounds the walk to the left; 8 entries per
            // read, then 32-entry block maxima
            int pg;
            {
                int wi = (e - 1) >> 3;
                const int bi = (e - 1) & 7;
                uint64_t hit = bytes_above(sW[wi], d) & (bi == 7 ? ~0ull : ((1ull << (8 * (bi + 1))) - 1ull));
                const int wlo = wi & ~3;
                while (!hit && wi > wlo) hit = bytes_above(sW[--wi], d);
                if (!hit) {
                    int blk = (wi >> 2) - 1;
                    while (sBM[blk] <= d) --blk;
                    wi = blk * 4 + 3;
                    while (!(hit = bytes_above(sW[wi], d))) --wi;
                }
                pg = wi * 8 + ((63 - __clzll(hit)) >> 3);
            }
            // NG: sD[m] = kTop bounds the walk to the right
            int ng;
            {
                int wi = (e + 1) >> 3;
                const int bi = (e + 1) & 7;
                uint64_t hit = bytes_above(sW[wi], d) & ~((1ull << (8 * bi)) - 1ull);
                const int whi = wi | 3;
                while (!hit && wi < whi) hit = bytes_above(sW[++wi], d);
                if (!hit) {
                    int blk = (wi >> 2) + 1;
                    while (sBM[blk] <= d) ++blk;
                    wi = blk * 4;
                    while (!(hit = bytes_above(sW[wi], d))) ++wi;
                }
                ng = wi * 8 + (__ffsll(static_cast<unsigned long long>(hit)) - 1) / 8;
            }
            const uint32_t R = uint32_t(ng - e), L = uint32_t(e - pg);
            atomicAdd(&sDiff[pg], R);
            atomicAdd(&sDiff[e], 0u - (R + L));
            atomicAdd(&sDiff[ng], L);
        }
        __syncthreads();
        // inclusive prefix sum of sDiff[0, m): kGsIPT consecutive entries per thread
        {
            const uint32_t base = uint32_t(tid) * kGsIPT;
            uint32_t loc[kGsIPT], run = 0;
#pragma unroll
            for (int q = 0; q < kGsIPT; ++q) {
                run += (base + q < m) ? sDiff[base + q] : 0u;
                loc[q] = run;
            }
            uint32_t tot;
            const uint32_t off = block_excl_scan<kGsThreads / 64>(run, sWave, tot);
#pragma unroll
            for (int q = 0; q < kGsIPT; ++q)
                if (base + q < m) sDiff[base + q] = loc[q] + off;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kGsIPT; ++k) {
            const uint32_t e = k * kGsThreads + tid;
            if (e >= m) continue;
            const uint64_t d = a + e + uint64_t(int64_t(int32_t(sDiff[e])));
            A.Xd[d] = A.Xs[a + e];
            A.Zd[d] = A.Zs[a + e];
            if (A.Ls) {
#pragma unroll
                for (int l = 0; l < LP; ++l) A.Ld[d * LP + l] = A.Ls[(a + e) * LP + l];
            }
            if constexpr (kRegC) {
#pragma unroll
                for (int l = 0; l < LP; ++l) Cd[d * LP + l] = cr[k][l];
            } else {
                const uint64_t p = a + e;
#pragma unroll 4
                for (int l = 0; l < LP; ++l) Cd[d * LP + l] = Cs[p * LP + l];
            }
        }
        __syncthreads();
    }
}

hipError_t launch_group_sort(const GroupSortArgs& a, int dtype, int lp, hipStream_t s, int grid) {
    if (a.xor_order) {
#define L_GSX(T, L) k_group_sort_xor<T, L><<<dim3(grid), dim3(kGsThreads), 0, s>>>(a)
        ORQA_DISPATCH(dtype, lp, L_GSX);
#undef L_GSX
        return hipGetLastError();
    }
#define L_GS(T, L) k_group_sort<T, L><<<dim3(grid), dim3(kGsThreads), 0, s>>>(a)
    ORQA_DISPATCH(dtype, lp, L_GS);
#undef L_GS
    return hipGetLastError();
}

hipError_t launch_sort_pass(const SortPassArgs& a, int ipt, int dtype, int lp, hipStream_t s, int grid) {
    if (a.w < 1 || a.w > 8) return hipErrorInvalidValue;
    if (ipt == 8) {
#define L_SP(T, L) k_sort_pass<T, L, 8><<<dim3(grid), dim3(kThreads), 0, s>>>(a)
        ORQA_DISPATCH(dtype, lp, L_SP);
#undef L_SP
    } else if (ipt == 16) {
#define L_SP(T, L) k_sort_pass<T, L, 16><<<dim3(grid), dim3(kThreads), 0, s>>>(a)
        ORQA_DISPATCH(dtype, lp, L_SP);
#undef L_SP
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_reduce(Ctrl* ctrl, int buf, const ulonglong2* X, const void* C, uint64_t cap, int mode,
                         double eps_pend, int mx, double* partial, double* out, int dtype, int lp, hipStream_t s) {
    if (mode == 0) k_prefix_len<<<1, 64, 0, s>>>(ctrl, buf, X, cap);
#define L_RD(T, L)                                                                                    \
    k_reduce_partial<T, L><<<dim3(kReduceBlocks), dim3(kThreads), 0, s>>>(ctrl, buf, static_cast<const T*>(C), \
                                                                          cap, mode, eps_pend, mx, partial); \
    k_reduce_final<L><<<1, 64, 0, s>>>(partial, kReduceBlocks, out)
    ORQA_DISPATCH(dtype, lp, L_RD);
#undef L_RD
    return hipGetLastError();
}

hipError_t launch_learned_estimate(Ctrl* ctrl, int buf, const void* C, const float* gscore, uint64_t cap,
                                   double eps_pend, double eps_learned, int mx, double* partial, int dtype, int lp,
                                   hipStream_t s) {
#define L_LE(T, L)                                                                                           \
    k_learned_partial<T, L><<<dim3(kReduceBlocks), dim3(kThreads), 0, s>>>(ctrl, buf, static_cast<const T*>(C), \
                                                                           gscore, cap, eps_pend, eps_learned, mx, \
                                                                           partial);                              \
    k_learned_final<L><<<1, 64, 0, s>>>(partial, kReduceBlocks, ctrl)
    ORQA_DISPATCH(dtype, lp, L_LE);
#undef L_LE
    return hipGetLastError();
}

hipError_t launch_prefix_len(Ctrl* ctrl, int buf, const ulonglong2* X, hipStream_t s) {
    k_prefix_len<<<1, 64, 0, s>>>(ctrl, buf, X, 0);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    k_fill_u64<<<dim3(256), dim3(256), 0, s>>>(p, v, n);
    return hipGetLastError();
}

}  // namespace orqa
