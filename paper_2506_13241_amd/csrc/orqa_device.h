// Device helpers for the gfx950 kernels: 128-bit key words, the virtual
// front/back array, wave/block scans and decoupled look-back.
#pragma once

#include "orqa_internal.h"

namespace orqa {

// ---------------------------------------------------------------- keys
// ulonglong2 holds a 128-bit mask: .x = bits 0..63, .y = bits 64..127.

__device__ __forceinline__ bool k_eq(const ulonglong2& a, const ulonglong2& b) {
    return a.x == b.x && a.y == b.y;
}
__device__ __forceinline__ bool k_lt(const ulonglong2& a, const ulonglong2& b) {
    return a.y < b.y || (a.y == b.y && a.x < b.x);
}
__device__ __forceinline__ bool k_le(const ulonglong2& a, const ulonglong2& b) { return !k_lt(b, a); }

// x mask with bit 0 cleared (the "H" part of an RX pairing block).
__device__ __forceinline__ ulonglong2 k_h(const ulonglong2& a) { return make_ulonglong2(a.x & ~1ull, a.y); }

__device__ __forceinline__ int k_popc_and(const ulonglong2& a, const ulonglong2& b) {
    return __popcll(a.x & b.x) + __popcll(a.y & b.y);
}

// Rotation of an n-bit mask (n <= 128) stored in two words.
__device__ __forceinline__ ulonglong2 rotl_n(ulonglong2 v, int r, int n) {
    if (r == 0) return v;
    unsigned __int128 w = (static_cast<unsigned __int128>(v.y) << 64) | v.x;
    unsigned __int128 mask = (n == 128) ? ~static_cast<unsigned __int128>(0)
                                        : ((static_cast<unsigned __int128>(1) << n) - 1);
    w = ((w << r) | (w >> (n - r))) & mask;
    return make_ulonglong2(static_cast<uint64_t>(w), static_cast<uint64_t>(w >> 64));
}

// Rotate right by one within n bits: bit 0 moves to bit n-1.
__device__ __forceinline__ ulonglong2 rotr1_n(ulonglong2 v, int n) {
    const uint64_t b0 = v.x & 1ull;
    ulonglong2 r = make_ulonglong2((v.x >> 1) | (v.y << 63), v.y >> 1);
    if (b0) {
        const int t = n - 1;
        if (t < 64) r.x |= 1ull << t;
        else r.y |= 1ull << (t - 64);
    }
    return r;
}

__device__ __forceinline__ uint64_t vphys(uint64_t i, uint64_t nf, uint64_t cap) {
    return i < nf ? i : cap - 1 - (i - nf);
}

// ---------------------------------------------------------------- wave / block
__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

// Exclusive scan over the 256 threads of a block.  s_wave: 4 words of LDS.
template <int NW = kThreads / 64>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* s_wave, uint32_t& total) {
    const int w = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(v);
    if (lane_id() == 63) s_wave[w] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        const uint32_t s = s_wave[i];
        off += (i < w) ? s : 0u;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return inc - v + off;
}

// ---------------------------------------------------------------- atomics
__device__ __forceinline__ uint64_t ld_acq(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_rel(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld32(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- look-back
// Status word: [63:40] epoch (24 bits) | [39:38] flag (1 aggregate, 2 inclusive)
// | [37:0] value.  Entries from another launch carry another epoch and read as
// "not ready", so status arrays never need clearing between launches.
constexpr uint64_t kValMask = (1ull << 38) - 1;
constexpr uint64_t kLookbackTicks = 200000000ull;  // ~2 s of the 100 MHz wall clock
constexpr int kLbPer = 1;                          // status words per lane per look-back round trip (wider windows measured slower)
constexpr int kLbWin = 64 * kLbPer;

__device__ __forceinline__ uint64_t st_pack(uint32_t ep, uint32_t fl, uint64_t v) {
    return (static_cast<uint64_t>(ep & 0xFFFFFFu) << 40) | (static_cast<uint64_t>(fl) << 38) | (v & kValMask);
}
__device__ __forceinline__ uint32_t st_flag(uint64_t s, uint32_t ep) {
    return (static_cast<uint32_t>(s >> 40) == (ep & 0xFFFFFFu)) ? static_cast<uint32_t>((s >> 38) & 3u) : 0u;
}

// Wave-parallel decoupled look-back for one channel (st indexed by tile with
// stride `stride`).  Must be called by all 64 lanes of one wave; returns the
// exclusive prefix of `tile` (uniform).  Publishes the aggregate first, so a
// tile never waits before its own aggregate is visible: every wait ends once
// the earlier tiles (which took their indices first) publish theirs.
// In two halves, so that a workgroup can publish a tile's aggregate, do other
// work and resolve the prefix later (each called by all 64 lanes of one
// wave; the aggregate is published before any wait, so every wait ends).
__device__ __forceinline__ void lookback_publish(uint64_t* st, uint64_t stride, uint32_t tile, uint32_t ep,
                                                 uint64_t agg) {
    if (lane_id() == 0) st_rel(st + tile * stride, st_pack(ep, tile == 0 ? 2u : 1u, agg));
}

__device__ __forceinline__ uint64_t lookback_resolve(uint64_t* st, uint64_t stride, uint32_t tile, uint32_t ep,
                                                     uint64_t agg, uint32_t* err) {
    const int lane = lane_id();
    if (tile == 0) return 0;
    uint64_t excl = 0;
    int64_t base = static_cast<int64_t>(tile) - 1;
    const uint64_t t0 = wall_clock64();
    bool timed_out = false;
    // Window of 64 * kLbPer predecessors per round trip: lane l holds distances
    // l*kLbPer .. l*kLbPer + kLbPer-1 (distance 0 is the nearest predecessor).
    while (true) {
        uint64_t v[kLbPer];
        int di = kLbWin, dr = kLbWin;
        while (true) {
            int fi_l = kLbPer, fr_l = kLbPer;
#pragma unroll
            for (int k = 0; k < kLbPer; ++k) {
                const int64_t j = base - (lane * kLbPer + k);
                v[k] = j >= 0 ? ld_acq(st + j * stride) : 0ull;
            }
#pragma unroll
            for (int k = kLbPer - 1; k >= 0; --k) {
                const int64_t j = base - (lane * kLbPer + k);
                const uint32_t fl = j >= 0 ? st_flag(v[k], ep) : 2u;  // before tile 0: inclusive 0
                if (fl == 2u) fi_l = k;
                if (fl == 0u) fr_l = k;
            }
            // Only the run from the nearest predecessor up to the first
            // inclusive prefix matters; tiles beyond it may still be loading.
            const uint64_t il = __ballot(fi_l < kLbPer);
            const uint64_t pl = __ballot(fr_l < kLbPer);
            if (il) {
                const int L = __ffsll(static_cast<unsigned long long>(il)) - 1;
                di = L * kLbPer + __shfl(fi_l, L, 64);
            }
            if (pl) {
                const int L = __ffsll(static_cast<unsigned long long>(pl)) - 1;
                dr = L * kLbPer + __shfl(fr_l, L, 64);
            }
            if (dr > di || dr == kLbWin) break;
            di = dr = kLbWin;
            if (__any(wall_clock64() - t0 > kLookbackTicks)) {
                timed_out = true;
                break;
            }
            __builtin_amdgcn_s_sleep(16);
        }
        if (timed_out) {
            if (lane == 0) atomicOr(err, kErrLookback);
            excl = 0;
            break;
        }
        uint64_t c = 0;
#pragma unroll
        for (int k = 0; k < kLbPer; ++k)
            if (lane * kLbPer + k <= di) c += v[k] & kValMask;
        excl += wave_sum_u64(c);
        if (di < kLbWin) break;
        base -= kLbWin;
    }
    if (lane == 0) st_rel(st + tile * stride, st_pack(ep, 2, excl + agg));
    return excl;
}

__device__ __forceinline__ uint64_t lookback_wave(uint64_t* st, uint64_t stride, uint32_t tile, uint32_t ep, uint64_t agg,
                                                  uint32_t* err) {
    lookback_publish(st, stride, tile, ep, agg);
    return lookback_resolve(st, stride, tile, ep, agg, err);
}

// Back-off between polls of the two-level look-back, in units of 64 clocks.
// Pollers of one prefix frontier all read the same few status lines, so a
// longer back-off relieves those lines more than it delays the poller
// (measured on the RX merge: 16 -> 40 is 3.5% faster, 100 slower again).
constexpr int kLb2Sleep = 40;

// Two-level decoupled look-back.  Tiles form groups of 64; the last tile of
// a group also publishes the group's aggregate (before its own look-back) and
// the group's inclusive prefix (after it) in gst[group].  A tile sums the
// tiles of its own group that precede it, then walks back over groups, 64
// groups (4096 tiles) per round trip: the inclusive prefixes no longer have to
// creep forward 64 tiles per round trip.
//
// It comes in two halves so that a workgroup can publish a tile's aggregate,
// do other work, and resolve the tile's prefix later: lb2_publish and
// lb2_resolve, each called by all 64 lanes of one wave.  Every wait is on
// tiles or groups that took their indices earlier, and both the aggregates
// and a group's aggregate (formed by the group's last tile in lb2_publish
// from its group's aggregates) are published before their tile waits for
// any prefix, so every wait ends as long as each tile's aggregate is
// published before its workgroup waits in lb2_resolve for a later tile.

// Publish the aggregate of `tile` (tile 0: its inclusive prefix); the last
// tile of a group then publishes the group's status.
__device__ __forceinline__ void lb2_publish(uint64_t* st, uint64_t* gst, uint32_t tile, uint32_t ep, uint64_t agg,
                                            uint32_t* err) {
    const int lane = lane_id();
    if (tile == 0) {
        if (lane == 0) st_rel(st, st_pack(ep, 2, agg));
        return;
    }
    if (lane == 0) st_rel(st + tile, st_pack(ep, 1, agg));
    if ((tile & 63u) != 63u) return;
    // Scanning the group from its end (lane 0 = this tile), the words up to
    // the first inclusive prefix give the group's inclusive prefix; with
    // none, all 64 aggregates give the group aggregate.  (A tile's word may
    // already hold its inclusive prefix instead of its aggregate, so the
    // scan stops there.)
    const uint64_t t0 = wall_clock64();
    uint64_t v;
    int fi = 64;
    while (true) {
        v = ld_acq(st + tile - lane);
        const uint32_t fl = st_flag(v, ep);
        const uint64_t incl = __ballot(fl == 2u);
        const uint64_t pend = __ballot(fl == 0u);
        fi = incl ? (__ffsll(static_cast<unsigned long long>(incl)) - 1) : 64;
        const int fr = pend ? (__ffsll(static_cast<unsigned long long>(pend)) - 1) : 64;
        if (fr > fi || fr == 64) break;
        if (__any(wall_clock64() - t0 > kLookbackTicks)) {
            if (lane == 0) atomicOr(err, kErrLookback);
            return;
        }
        __builtin_amdgcn_s_sleep(kLb2Sleep);
    }
    const uint64_t gsum = wave_sum_u64(lane <= fi ? (v & kValMask) : 0ull);
    if (lane == 0) st_rel(gst + (tile >> 6), st_pack(ep, fi < 64 ? 2u : 1u, gsum));
}

// Exclusive prefix of `tile` (uniform), whose aggregate `agg` lb2_publish has
// published; publishes the tile's (and, for the last tile of a group, the
// group's) inclusive prefix.
__device__ __forceinline__ uint64_t lb2_resolve(uint64_t* st, uint64_t* gst, uint32_t tile, uint32_t ep,
                                                uint64_t agg, uint32_t* err) {
    const int lane = lane_id();
    if (tile == 0) return 0;
    const uint32_t grp = tile >> 6, first = grp << 6;
    const bool last_in_group = (tile & 63u) == 63u;
    const uint64_t t0 = wall_clock64();
    bool timed_out = false;
    uint64_t excl = 0;
    bool done = false;
    // ---- within the group: tiles first .. tile-1, nearest first
    if (tile > first) {
        const int64_t j = int64_t(tile) - 1 - lane;
        const bool in = j >= int64_t(first);
        uint64_t v = 0;
        int fi = 64;
        while (true) {
            uint32_t fl = 1;  // lanes outside the group: ready, value 0
            v = 0;
            if (in) {
                v = ld_acq(st + j);
                fl = st_flag(v, ep);
            }
            const uint64_t incl = __ballot(in && fl == 2u);
            const uint64_t pend = __ballot(fl == 0u);
            fi = incl ? (__ffsll(static_cast<unsigned long long>(incl)) - 1) : 64;
            const int fr = pend ? (__ffsll(static_cast<unsigned long long>(pend)) - 1) : 64;
            if (fr > fi || fr == 64) break;
            if (__any(wall_clock64() - t0 > kLookbackTicks)) {
                timed_out = true;
                break;
            }
            __builtin_amdgcn_s_sleep(kLb2Sleep);
        }
        if (!timed_out) {
            excl += wave_sum_u64((in && lane <= fi) ? (v & kValMask) : 0ull);
            done = fi < 64;
        }
    }
    // ---- earlier groups, 64 per round trip (group 0 always publishes an
    // inclusive prefix: its scan reaches tile 0, which is inclusive at once)
    if (!timed_out && !done && grp > 0) {
        int64_t base = int64_t(grp) - 1;
        while (true) {
            const int64_t g = base - lane;
            uint64_t v = 0;
            int fi = 64;
            uint64_t incl = 0;
            while (true) {
                uint32_t fl = 2;  // before group 0: inclusive 0
                v = 0;
                if (g >= 0) {
                    v = ld_acq(gst + g);
                    fl = st_flag(v, ep);
                }
                incl = __ballot(fl == 2u);
                const uint64_t pend = __ballot(fl == 0u);
                fi = incl ? (__ffsll(static_cast<unsigned long long>(incl)) - 1) : 64;
                const int fr = pend ? (__ffsll(static_cast<unsigned long long>(pend)) - 1) : 64;
                if (fr > fi || fr == 64) break;
                if (__any(wall_clock64() - t0 > kLookbackTicks)) {
                    timed_out = true;
                    break;
                }
                __builtin_amdgcn_s_sleep(kLb2Sleep);
            }
            if (timed_out) break;
            excl += wave_sum_u64(lane <= fi ? (v & kValMask) : 0ull);
            if (incl) break;
            base -= 64;
        }
    }
    if (timed_out) {
        if (lane == 0) atomicOr(err, kErrLookback);
        excl = 0;
    }
    if (lane == 0) {
        st_rel(st + tile, st_pack(ep, 2, excl + agg));
        if (last_in_group) st_rel(gst + grp, st_pack(ep, 2, excl + agg));
    }
    return excl;
}

// Both halves back to back: the exclusive prefix of `tile` (uniform).
__device__ __forceinline__ uint64_t lookback_wave2(uint64_t* st, uint64_t* gst, uint32_t tile, uint32_t ep,
                                                   uint64_t agg, uint32_t* err) {
    lb2_publish(st, gst, tile, ep, agg, err);
    return lb2_resolve(st, gst, tile, ep, agg, err);
}

// Single-thread look-back (one channel per thread, used by the radix sort with
// one thread per digit).
__device__ __forceinline__ uint64_t lookback_thread(uint64_t* st, uint64_t stride, uint32_t tile, uint32_t ep, uint64_t agg,
                                    uint32_t* err) {
    if (tile == 0) {
        st_rel(st, st_pack(ep, 2, agg));
        return 0;
    }
    st_rel(st + tile * stride, st_pack(ep, 1, agg));
    uint64_t excl = 0;
    int64_t j = static_cast<int64_t>(tile) - 1;
    const uint64_t t0 = wall_clock64();
    while (j >= 0) {
        const uint64_t v = ld_acq(st + j * stride);
        const uint32_t fl = st_flag(v, ep);
        if (fl != 0u) {
            excl += v & kValMask;
            if (fl == 2u) break;
            --j;
        } else {
            if (wall_clock64() - t0 > kLookbackTicks) {
                atomicOr(err, kErrLookback);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
    }
    st_rel(st + tile * stride, st_pack(ep, 2, excl + agg));
    return excl;
}

// Dynamic tile acquisition for persistent look-back kernels.
__device__ __forceinline__ uint32_t acquire_tile(Ctrl* ctrl, uint32_t* s_tile) {
    // Tiles are dealt round-robin to S = min(kTileStreams, gridDim.x) streams
    // of workgroups (stream = blockIdx modulo S), each with a counter of its
    // own, so no single address takes every acquisition.  Every stream has a
    // workgroup, and a stream takes its tiles in increasing order.
    if (threadIdx.x == 0) {
        const uint32_t S = gridDim.x < kTileStreams ? gridDim.x : kTileStreams;
        const uint32_t st = blockIdx.x % S;
        *s_tile = atomicAdd(&ctrl->tile_ctr[st][0], 1u) * S + st;
    }
    __syncthreads();
    const uint32_t t = *s_tile;
    __syncthreads();
    return t;
}

// Exit protocol of every look-back kernel: the last workgroup to finish resets
// the tile and done counters and advances the epoch.  Returns true in the one
// thread that performs the reset (for extra end-of-launch bookkeeping).
// Counts the workgroup done; the last one to finish gets true.  Every wave
// first waits for its own memory operations to complete.  What a last
// workgroup reads of the others' writes (the error bits, the maxima, the
// output sizes) is written with agent-scope atomics, which complete at the
// device's point of coherence, so that wait orders them before the count and
// no device-scope fence is needed here: such a fence writes back and
// invalidates the XCD's L2, and one per workgroup at the end of a launch
// stalls every workgroup still running.
__device__ __forceinline__ bool finish_launch(Ctrl* ctrl) {
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    bool last = false;
    if (threadIdx.x == 0) {
        const uint32_t d = atomicAdd(&ctrl->done_counter, 1u);
        if (d == gridDim.x - 1) {
            __threadfence();
            for (uint32_t i = 0; i < kTileStreams; ++i)
                __hip_atomic_store(&ctrl->tile_ctr[i][0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctrl->tile_counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctrl->done_counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctrl->epoch, ctrl->epoch + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            last = true;
        }
    }
    return last;
}

// ---------------------------------------------------------------- coefficient arithmetic
// Binary64: plain products and one sum (no contraction: -ffp-contract=off).
// Binary32: error-free products with fmaf plus two-sum, rounded once.

struct F32x2 {
    float hi, lo;
};

__device__ __forceinline__ F32x2 two_prod(float a, float b) {
    const float p = a * b;
    return {p, fmaf(a, b, -p)};
}
__device__ __forceinline__ F32x2 two_sum(float a, float b) {
    const float s = a + b;
    const float bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
// c * (hi + lo) as an unevaluated pair.
__device__ __forceinline__ F32x2 mul_split(float c, float hi, float lo) {
    F32x2 p = two_prod(c, hi);
    p.lo = fmaf(c, lo, p.lo);
    return p;
}

template <typename CT>
struct Arith;

template <>
struct Arith<double> {
    __device__ static __forceinline__ double scale_c(const GateTrig& g, int a, double c) { return g.cs[a] * c; }
    __device__ static __forceinline__ double scale_s(const GateTrig& g, int a, double c, bool neg) {
        const double s = neg ? -g.sn[a] : g.sn[a];
        return s * c;
    }
    __device__ static __forceinline__ double pair(const GateTrig& g, int a, double cp, double cc, bool neg) {
        const double s = neg ? -g.sn[a] : g.sn[a];
        const double x = g.cs[a] * cp;
        const double y = s * cc;
        return x + y;
    }
};

template <>
struct Arith<float> {
    __device__ static __forceinline__ float scale_c(const GateTrig& g, int a, float c) {
        const F32x2 p = mul_split(c, g.cs_hi[a], g.cs_lo[a]);
        return p.hi + p.lo;
    }
    __device__ static __forceinline__ float scale_s(const GateTrig& g, int a, float c, bool neg) {
        const float h = neg ? -g.sn_hi[a] : g.sn_hi[a];
        const float l = neg ? -g.sn_lo[a] : g.sn_lo[a];
        const F32x2 p = mul_split(c, h, l);
        return p.hi + p.lo;
    }
    __device__ static __forceinline__ float pair(const GateTrig& g, int a, float cp, float cc, bool neg) {
        const float h = neg ? -g.sn_hi[a] : g.sn_hi[a];
        const float l = neg ? -g.sn_lo[a] : g.sn_lo[a];
        const F32x2 p = mul_split(cp, g.cs_hi[a], g.cs_lo[a]);
        const F32x2 q = mul_split(cc, h, l);
        const F32x2 s = two_sum(p.hi, q.hi);
        return s.hi + (s.lo + (p.lo + q.lo));
    }
};

template <typename CT>
__device__ __forceinline__ double absd(CT v) {
    return fabs(static_cast<double>(v));
}

__device__ __forceinline__ double bits_to_d(uint64_t b) { return __longlong_as_double(static_cast<long long>(b)); }
__device__ __forceinline__ uint64_t d_to_bits(double d) { return static_cast<uint64_t>(__double_as_longlong(d)); }

}  // namespace orqa
