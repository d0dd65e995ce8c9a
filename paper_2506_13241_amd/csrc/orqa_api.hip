// Host engine and C ABI of the gfx950 Pauli-propagation library.
#include <algorithm>
#include <cstdint>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/orqa.h"
#include "orqa_internal.h"
#include "orqa_scorer.h"

using namespace orqa;

namespace {

thread_local std::string g_last_error = "ok";

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

}  // namespace

namespace orqa {
int api_fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}
int scorer_alloc(ScorerDev* d);
void scorer_free(ScorerDev* d);
int scorer_copy(ScorerDev* dst, const ScorerDev* src, hipStream_t s);
const ScorerDev* scorer_dev(const ps_scorer* s);
}  // namespace orqa

namespace {

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t _e = (expr);                                                                \
        if (_e != hipSuccess) return fail(PS_ERR_HIP, "%s: %s", #expr, hipGetErrorString(_e)); \
    } while (0)

int lanes_pad(int L) {
    int p = 1;
    while (p < L) p <<= 1;
    return p;
}

// Exact trigonometry at multiples of pi/2 (within 1e-12*max(1,|theta|)).
// Returns the multiple k mod 4, or -1 for a generic angle.
int classify(double theta, double* c, double* s) {
    const double half_pi = M_PI / 2.0;
    const double k = std::nearbyint(theta / half_pi);
    if (std::fabs(theta - k * half_pi) <= 1e-12 * std::fmax(1.0, std::fabs(theta))) {
        long m = static_cast<long>(std::fmod(k, 4.0));
        if (m < 0) m += 4;
        static const double C[4] = {1.0, 0.0, -1.0, 0.0};
        static const double S[4] = {0.0, 1.0, 0.0, -1.0};
        *c = C[m];
        *s = S[m];
        return static_cast<int>(m);
    }
    *c = std::cos(theta);
    *s = std::sin(theta);
    return -1;
}

void split_f32(double v, float* hi, float* lo) {
    *hi = static_cast<float>(v);
    *lo = static_cast<float>(v - static_cast<double>(*hi));
}

struct U128 {
    uint64_t lo, hi;
};

U128 rotr_host(U128 v, int r, int n) {
    r %= n;
    if (r == 0) return v;
    unsigned __int128 w = (static_cast<unsigned __int128>(v.hi) << 64) | v.lo;
    unsigned __int128 mask = (n == 128) ? ~static_cast<unsigned __int128>(0)
                                        : ((static_cast<unsigned __int128>(1) << n) - 1);
    w = ((w >> r) | (w << (n - r))) & mask;
    return {static_cast<uint64_t>(w), static_cast<uint64_t>(w >> 64)};
}
U128 rotl_host(U128 v, int r, int n) { return rotr_host(v, (n - (r % n)) % n, n); }

enum StageKind { ST_RX = 0, ST_CLIFF = 1, ST_GEN = 2 };

struct Stage {
    StageKind kind;
    size_t gate_first, gate_count;  // gates of the layer covered by this stage
    GateTrig trig;                  // RX, general
    int qubit;                      // RX
    ps_pauli gen;                   // general
    std::vector<CliffGen> gens;     // Clifford run
    bool needs_sort;
};

}  // namespace

struct ps_handle {
    int nq = 0, L = 1, LP = 1, dtype = PS_F64;
    int dev = 0;        // HIP device current at creation (holds the buffers)
    // look-back launches since the status words were last cleared; the device
    // epoch equals 1 + this count, and the words are cleared before it reaches
    // 2^24 (the width of the epoch tag in a status word)
    uint64_t lb_count = 0;
    size_t csize = 8;  // bytes per coefficient row
    size_t cap = 0;
    Buf buf[2] = {};
    uint32_t* rank[2] = {nullptr, nullptr};
    Ctrl* ctrl = nullptr;
    TileDesc* desc = nullptr;  // RX tile boundaries (written and read by each RX launch)
    size_t desc_words = 0;     // desc as 64-bit words (each tagged with a launch epoch)
    uint64_t* status = nullptr;
    size_t status_words = 0;
    uint64_t max_tiles = 0;
    uint32_t* hist = nullptr;
    uint32_t* digit_base = nullptr;
    double* partial = nullptr;
    double* red_out = nullptr;
    CliffGen* cgens = nullptr;
    int cur = 0;        // state buffer holding the operator
    int mx = 0;         // max slot of the operator
    double pend = -1.0; // pending truncation eps of the operator (<= 0: none)
    int xrot = 0;       // stored x = x rotated right by xrot
    hipStream_t stream = nullptr;
    int grid = 1024;
    int rx_grid = 1024;  // RX merge workgroups: what the CUs hold at once (at most grid)
    bool rx_no_prologue = false;  // tiles find their own boundaries (pauli_sum_set_rx_boundary_prologue)
    size_t gates_applied = 0;
    uint64_t n_host = 0;  // size after the last synchronisation
    bool broken = false;
    // learned truncation: its threshold is learned_ratio * rel_eps; with
    // learned_tol > 0 a pass whose estimated learned error exceeds it falls
    // back to the magnitude rule
    double learned_ratio = 1.0, learned_tol = 0.0;
    bool has_scorer = false;
    ScorerDev scorer{};
    float* gscore = nullptr;  // cap floats
    // measurement: event pairs around launches, folded into host totals at syncs
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> ev_kind;  // 0 rx merge, 1 clifford/compaction, 2 sort pass, 3 learned scorer
    size_t ev_used = 0;
    double ms[4] = {0, 0, 0, 0};
    double sort_passes = 0, sort_elems = 0, gates = 0;
    // captured runs of RX stages (see run_rx_graph)
    bool graphs = false;
    hipStream_t cap_stream = nullptr;
    uint64_t alloc_gen = 0;  // bumped whenever device buffers move
    struct GraphEntry {
        uint64_t key;
        size_t n_stages;
        hipGraphExec_t exec;
    };
    std::vector<GraphEntry> graph_cache;
    double graph_replays = 0, graph_captures = 0;
    // general gates with x_J = 0: after a group sort that overflowed, the next
    // gs_skip such gates go straight to the radix sort
    int gs_skip = 0;
    // radix-sort configuration: forced by pauli_sum_set_sort_config, or tuned
    // online (each candidate timed once per key kind and size class, then
    // the fastest kept); every configuration gives the same result
    int sort_force = -1;  // candidate index, -1: tune
    float sort_ns[2][64][6] = {};  // ns per string, 0: not tried yet
    hipEvent_t sort_ev[2] = {nullptr, nullptr};
    int sort_last = 0;
    double radix_sorts = 0;
    // binary32 general gates: low words of the branch's products, one array
    // per state buffer (allocated with the auxiliaries once the handle has
    // run such a gate); lo_live while a general gate's entries carry them
    bool has_lo = false;
    bool lo_live = false;
    float* lo[2] = {nullptr, nullptr};
    // general gates: runs of the last branch (-1: unsorted output, radix
    // sort), the merge-path split buffer and the count of run merges
    int gen_run_bits = -1;
    uint64_t* msplit = nullptr;
    size_t msplit_words = 0;
    double run_merges = 0;
};

namespace {

size_t coef_bytes(const ps_handle* h) { return h->csize; }

// Device memory of the handle comes in three parts so that growing never holds
// more than the kept state buffer besides the new allocation: the two state
// buffers (keys and coefficients, `cap` strings each) and the per-capacity
// auxiliaries (rank arrays, tile descriptors, look-back status words, and the
// learned-score array when a scorer is loaded).
struct Aux {
    uint32_t* rank[2] = {nullptr, nullptr};
    TileDesc* desc = nullptr;
    size_t desc_words = 0;
    uint64_t* status = nullptr;
    size_t status_words = 0;
    uint64_t max_tiles = 0;
    float* gscore = nullptr;
    float* lo[2] = {nullptr, nullptr};
};

bool grab(void** p, size_t bytes) {
    if (hipMalloc(p, bytes ? bytes : 16) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return false;
    }
    return true;
}

void free_state(Buf* b) {
    if (b->X) (void)hipFree(b->X);
    if (b->Z) (void)hipFree(b->Z);
    if (b->C) (void)hipFree(b->C);
    *b = {};
}

bool alloc_state(ps_handle* h, size_t cap, Buf* b) {
    *b = {};
    if (grab(reinterpret_cast<void**>(&b->X), cap * sizeof(ulonglong2)) &&
        grab(reinterpret_cast<void**>(&b->Z), cap * sizeof(ulonglong2)) && grab(&b->C, cap * coef_bytes(h)))
        return true;
    free_state(b);
    return false;
}

void free_aux(Aux* a) {
    void* ps[] = {a->rank[0], a->rank[1], a->desc, a->status, a->gscore, a->lo[0], a->lo[1]};
    for (void* p : ps)
        if (p) (void)hipFree(p);
    *a = Aux{};
}

bool alloc_aux(ps_handle* h, size_t cap, bool with_score, Aux* a) {
    *a = Aux{};
    const uint64_t mt = cap / kRxTile + 4;
    const uint64_t st_tiles = cap / kCompactTile + 4;
    const uint64_t sort_tiles = cap / kSortTile + 4;
    const uint64_t tiles = std::max(mt, st_tiles);
    // per channel: one word per tile, then one per group of 64 tiles (RX merge)
    const size_t words = std::max<size_t>(2 * tiles + 2 * (tiles / 64 + 2), 256 * sort_tiles);
    bool ok = grab(reinterpret_cast<void**>(&a->rank[0]), cap * sizeof(uint32_t)) &&
              grab(reinterpret_cast<void**>(&a->rank[1]), cap * sizeof(uint32_t)) &&
              grab(reinterpret_cast<void**>(&a->desc), (mt + 2) * sizeof(TileDesc)) &&
              grab(reinterpret_cast<void**>(&a->status), words * sizeof(uint64_t));
    if (ok && with_score) ok = grab(reinterpret_cast<void**>(&a->gscore), cap * sizeof(float));
    if (ok && h->has_lo)
        ok = grab(reinterpret_cast<void**>(&a->lo[0]), cap * h->LP * sizeof(float)) &&
             grab(reinterpret_cast<void**>(&a->lo[1]), cap * h->LP * sizeof(float));
    // status words start from a zero epoch tag the kernels never use (epoch starts at 1)
    if (ok) ok = hipMemsetAsync(a->status, 0, words * sizeof(uint64_t), h->stream) == hipSuccess;
    if (ok) ok = hipMemsetAsync(a->desc, 0, (mt + 2) * sizeof(TileDesc), h->stream) == hipSuccess;
    if (!ok) {
        free_aux(a);
        return false;
    }
    a->status_words = words;
    a->desc_words = (mt + 2) * sizeof(TileDesc) / sizeof(uint64_t);
    a->max_tiles = std::max(mt, st_tiles);
    return true;
}

Aux take_aux(ps_handle* h) {
    Aux a;
    a.rank[0] = h->rank[0];
    a.rank[1] = h->rank[1];
    a.desc = h->desc;
    a.desc_words = h->desc_words;
    a.status = h->status;
    a.status_words = h->status_words;
    a.max_tiles = h->max_tiles;
    a.gscore = h->gscore;
    a.lo[0] = h->lo[0];
    a.lo[1] = h->lo[1];
    h->lo[0] = h->lo[1] = nullptr;
    h->rank[0] = h->rank[1] = nullptr;
    h->desc = nullptr;
    h->status = nullptr;
    h->gscore = nullptr;
    return a;
}

void put_aux(ps_handle* h, const Aux& a) {
    h->rank[0] = a.rank[0];
    h->rank[1] = a.rank[1];
    h->desc = a.desc;
    h->desc_words = a.desc_words;
    h->status = a.status;
    h->status_words = a.status_words;
    h->max_tiles = a.max_tiles;
    h->gscore = a.gscore;
    h->lo[0] = a.lo[0];
    h->lo[1] = a.lo[1];
}

void free_buffers(ps_handle* h) {
    free_state(&h->buf[0]);
    free_state(&h->buf[1]);
    Aux a = take_aux(h);
    free_aux(&a);
}

// Allocate both state buffers and the auxiliaries for `cap` strings.  On
// failure nothing is leaked and PS_ERR_CAPACITY is returned.
int alloc_buffers(ps_handle* h, size_t cap) {
    Aux a;
    if (!alloc_state(h, cap, &h->buf[0]) || !alloc_state(h, cap, &h->buf[1]) ||
        !alloc_aux(h, cap, h->has_scorer, &a)) {
        free_state(&h->buf[0]);
        free_state(&h->buf[1]);
        return fail(PS_ERR_CAPACITY, "hipMalloc failed for capacity %zu strings", cap);
    }
    put_aux(h, a);
    return PS_OK;
}

int ev_collect(ps_handle* h);

int read_ctrl(ps_handle* h, Ctrl* c) {
    HIP_TRY(hipMemcpyAsync(c, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return ev_collect(h);
}

// ---------------------------------------------------------------- timing
int ev_begin(ps_handle* h, int kind, size_t* slot) {
    *slot = SIZE_MAX;
    if (!h->timing) return PS_OK;
    if (h->ev_used + 2 > h->ev_pool.size()) {
        // timing-only events: no system-scope fence (cache writeback and
        // invalidate) when they complete; they are read after a stream
        // synchronisation
        for (int i = 0; i < 64; ++i) {
            hipEvent_t e;
            HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
            h->ev_pool.push_back(e);
        }
        h->ev_kind.resize(h->ev_pool.size() / 2);
    }
    *slot = h->ev_used;
    h->ev_kind[h->ev_used / 2] = kind;
    HIP_TRY(hipEventRecord(h->ev_pool[h->ev_used], h->stream));
    h->ev_used += 2;
    return PS_OK;
}
int ev_end(ps_handle* h, size_t slot) {
    if (slot == SIZE_MAX) return PS_OK;
    HIP_TRY(hipEventRecord(h->ev_pool[slot + 1], h->stream));
    return PS_OK;
}
// Fold recorded event pairs into the totals (the stream must be synchronised).
int ev_collect(ps_handle* h) {
    for (size_t i = 0; i + 1 < h->ev_used; i += 2) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, h->ev_pool[i], h->ev_pool[i + 1]));
        h->ms[h->ev_kind[i / 2]] += ms;
    }
    h->ev_used = 0;
    return PS_OK;
}

void drop_graphs(ps_handle* h);

// Grow capacity to at least `need`, keeping state buffer `keep` (front and back
// runs) and its sizes; the other buffer's contents are discarded.  Everything
// but the kept buffer is released first, so the peak is the kept buffer plus
// the new allocation.  If no larger capacity can be allocated the handle is
// restored at its old capacity and PS_ERR_CAPACITY returned.
int grow(ps_handle* h, int keep, uint64_t need) {
    Ctrl c;
    int rc = read_ctrl(h, &c);
    if (rc) return rc;
    drop_graphs(h);  // captured launches point at the buffers about to move
    h->alloc_gen += 1;
    free_state(&h->buf[1 - keep]);
    {
        Aux old = take_aux(h);
        free_aux(&old);
    }
    const size_t want[3] = {std::max<size_t>(need + need / 4 + 1024, h->cap + h->cap / 2), need + 1024, h->cap};
    size_t ncap = 0;
    Buf nout{}, nkeep{};
    Aux na;
    for (size_t cap : want) {
        if (cap < need && cap != h->cap) continue;
        if (!alloc_state(h, cap, &nout)) continue;
        if (!alloc_aux(h, cap, h->has_scorer, &na)) {
            free_state(&nout);
            continue;
        }
        if (cap != h->cap && !alloc_state(h, cap, &nkeep)) {
            free_state(&nout);
            free_aux(&na);
            continue;
        }
        ncap = cap;
        break;
    }
    if (ncap == 0) {
        h->broken = true;
        return fail(PS_ERR_CAPACITY, "hipMalloc failed while restoring capacity %zu (handle is no longer usable)",
                    h->cap);
    }
    h->buf[1 - keep] = nout;
    put_aux(h, na);
    if (ncap == h->cap) {
        HIP_TRY(hipStreamSynchronize(h->stream));
        return fail(PS_ERR_CAPACITY, "hipMalloc failed for capacity %zu strings (kept capacity %zu)",
                    size_t(need + need / 4 + 1024), h->cap);
    }
    const uint64_t f = c.nf[keep], b = c.nb[keep];
    const size_t cb = coef_bytes(h);
    auto cpy = [&](void* dst, const void* src, size_t bytes) -> hipError_t {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, h->stream) : hipSuccess;
    };
    const Buf& o = h->buf[keep];
    HIP_TRY(cpy(nkeep.X, o.X, f * sizeof(ulonglong2)));
    HIP_TRY(cpy(nkeep.Z, o.Z, f * sizeof(ulonglong2)));
    HIP_TRY(cpy(nkeep.C, o.C, f * cb));
    HIP_TRY(cpy(nkeep.X + (ncap - b), o.X + (h->cap - b), b * sizeof(ulonglong2)));
    HIP_TRY(cpy(nkeep.Z + (ncap - b), o.Z + (h->cap - b), b * sizeof(ulonglong2)));
    HIP_TRY(cpy(static_cast<char*>(nkeep.C) + (ncap - b) * cb, static_cast<const char*>(o.C) + (h->cap - b) * cb,
                b * cb));
    HIP_TRY(hipStreamSynchronize(h->stream));
    free_state(&h->buf[keep]);
    h->buf[keep] = nkeep;
    h->cap = ncap;
    return PS_OK;
}

// Clear a kernel-raised capacity error so the failed stage can be re-run: the
// failed stage left its input untouched; its output max slot is reset.
int clear_error(ps_handle* h, int mx_out) {
    Ctrl c;
    int rc = read_ctrl(h, &c);
    if (rc) return rc;
    c.err = 0;
    c.need = 0;
    for (int a = 0; a < kMaxLanes; ++a) c.maxbits[mx_out][a] = 0;
    HIP_TRY(hipMemcpyAsync(h->ctrl, &c, sizeof(Ctrl), hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return PS_OK;
}

int check_no_error(ps_handle* h, const char* what) {
    Ctrl c;
    int rc = read_ctrl(h, &c);
    if (rc) return rc;
    if (c.err & kErrLookback) {
        h->broken = true;
        return fail(PS_ERR_DEVICE, "%s: look-back wait timed out (handle is no longer usable)", what);
    }
    if (c.err) return fail(PS_ERR_DEVICE, "%s: kernel error bits 0x%x", what, c.err);
    h->n_host = c.nf[h->cur] + c.nb[h->cur];
    return PS_OK;
}

// Status words carry the low 24 bits of the launch epoch; a word written 2^24
// look-back launches earlier and not since would read as current.  Before the
// epoch gets there, clear every status word and restart the epoch at 1.  Must
// be called before enqueueing `k` look-back launches, outside stream capture.
constexpr uint64_t kEpochLimit = (uint64_t(1) << 24) - 2;

int lb_reserve(ps_handle* h, uint64_t k) {
    if (h->lb_count + k < kEpochLimit) {
        h->lb_count += k;
        return PS_OK;
    }
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(launch_fill_u64(h->status, 0ull, h->status_words, h->stream));
    HIP_TRY(launch_fill_u64(reinterpret_cast<uint64_t*>(h->desc), 0ull, h->desc_words, h->stream));
    const uint32_t one = 1;
    HIP_TRY(hipMemcpyAsync(&h->ctrl->epoch, &one, sizeof one, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->lb_count = k;
    return PS_OK;
}

#define LB_RESERVE(h, k)                \
    do {                                \
        const int _rc = lb_reserve(h, k); \
        if (_rc) return _rc;            \
    } while (0)

// ---------------------------------------------------------------- stages

// A Clifford run's generators for the pass: weight-2 generators grouped by
// qubit offset (one slot per lower qubit and offset; a repeated pair, or more
// offsets than kMaxCliffGroups, stays in the one-by-one list with every other
// generator).  The generators commute, so the grouping does not change the
// product.
void group_cliff_gens(const std::vector<CliffGen>& gens, std::vector<CliffGroup>& groups,
                      std::vector<CliffGen>& rest) {
    groups.clear();
    rest.clear();
    for (const CliffGen& g : gens) {
        const int w = __builtin_popcountll(g.z0) + __builtin_popcountll(g.z1);
        bool placed = false;
        if (w == 2) {
            const int a = g.z0 ? __builtin_ctzll(g.z0) : 64 + __builtin_ctzll(g.z1);
            const uint64_t hi0 = g.z0 & ~(a < 64 ? (1ull << a) : 0ull);
            const uint64_t hi1 = g.z1 & ~(a >= 64 ? (1ull << (a - 64)) : 0ull);
            const int b = hi0 ? __builtin_ctzll(hi0) : 64 + __builtin_ctzll(hi1);
            const uint32_t d = uint32_t(b - a);
            CliffGroup* grp = nullptr;
            for (CliffGroup& c : groups)
                if (c.d == d) grp = &c;
            if (!grp && groups.size() < size_t(kMaxCliffGroups)) {
                groups.push_back(CliffGroup{0, 0, 0, 0, d, 0});
                grp = &groups.back();
            }
            const uint64_t m0 = a < 64 ? (1ull << a) : 0ull, m1 = a >= 64 ? (1ull << (a - 64)) : 0ull;
            if (grp && !((grp->k0 | grp->n0) & m0) && !((grp->k1 | grp->n1) & m1)) {
                if (g.kodd) {
                    grp->k0 |= m0;
                    grp->k1 |= m1;
                }
                if (g.neg) {
                    grp->n0 |= m0;
                    grp->n1 |= m1;
                }
                placed = true;
            }
        }
        if (!placed) rest.push_back(g);
    }
}

int enqueue_compact(ps_handle* h, int in, int out, int mx_in, int mx_out, double eps_in, const CliffGen* gens,
                    int ngens, bool with_rank, int gate_count = 0, double eps_learned = -1.0,
                    const CliffGroup* groups = nullptr, int ngroups = 0, bool groups_neg_is_k = false) {
    const bool learned = eps_learned > 0.0;
    if (learned) {  // score every input string, then the compaction applies the learned rule
        ScorerFwdArgs f{};
        f.net = h->scorer;
        f.X = h->buf[in].X;
        f.Z = h->buf[in].Z;
        f.nf_ptr = &h->ctrl->nf[in];
        f.nb_ptr = &h->ctrl->nb[in];
        f.cap = h->cap;
        f.xrot = h->xrot;
        f.nq = h->nq;
        f.y_out = h->gscore;
        f.counters = &h->ctrl->aux[0];
        size_t slot;
        int rc = ev_begin(h, 3, &slot);
        if (rc) return rc;
        HIP_TRY(launch_scorer_forward(f, h->stream, h->grid / 2));  // two 512-thread workgroups per CU
        rc = ev_end(h, slot);
        if (rc) return rc;
        HIP_TRY(launch_learned_estimate(h->ctrl, in, h->buf[in].C, h->gscore, h->cap, eps_in, eps_learned, mx_in,
                                        h->partial, h->dtype, h->LP, h->stream));
    }
    CompactArgs a{};
    a.ctrl = h->ctrl;
    a.in_buf = in;
    a.out_buf = out;
    a.mx_in = mx_in;
    a.mx_out = mx_out;
    a.Xin = h->buf[in].X;
    a.Zin = h->buf[in].Z;
    a.Cin = h->buf[in].C;
    a.Xout = h->buf[out].X;
    a.Zout = h->buf[out].Z;
    a.Cout = h->buf[out].C;
    a.rank_out = with_rank ? h->rank[out] : nullptr;
    a.cap = h->cap;
    a.status = h->status;
    a.max_tiles = h->max_tiles;
    a.eps_in = eps_in;
    a.nq = h->nq;
    a.xrot = h->xrot;
    a.gens = gens;
    a.ngens = ngens;
    a.groups = groups;
    a.ngroups = ngroups;
    a.groups_neg_is_k = groups_neg_is_k ? 1 : 0;
    a.gate_count = gate_count;
    a.gscore = learned ? h->gscore : nullptr;
    a.eps_learned = learned ? eps_learned : 0.0;
    a.learned_tol = h->learned_tol;
    size_t slot;
    int rc = ev_begin(h, 1, &slot);
    if (rc) return rc;
    LB_RESERVE(h, 1);
    HIP_TRY(launch_compact(a, h->dtype, h->LP, h->stream, h->grid));
    return ev_end(h, slot);
}

int enqueue_rx(ps_handle* h, int in, int out, int mx_in, int mx_out, double eps_in, const GateTrig& g,
               hipStream_t stream = nullptr, bool timed = true, bool capturing = false) {
    if (!stream) stream = h->stream;
    RxArgs a{};
    a.ctrl = h->ctrl;
    a.in_buf = in;
    a.out_buf = out;
    a.mx_in = mx_in;
    a.mx_out = mx_out;
    a.Xin = h->buf[in].X;
    a.Zin = h->buf[in].Z;
    a.Cin = h->buf[in].C;
    a.Xout = h->buf[out].X;
    a.Zout = h->buf[out].Z;
    a.Cout = h->buf[out].C;
    a.cap = h->cap;
    a.desc = h->desc;
    a.status = h->status;
    a.max_tiles = h->max_tiles;
    a.eps_in = eps_in;
    a.nq = h->nq;
    a.no_prologue = h->rx_no_prologue ? 1 : 0;
    if (!capturing) LB_RESERVE(h, 1);  // a captured run reserves its launches at replay
    size_t slot = SIZE_MAX;
    if (timed) {
        int rc = ev_begin(h, 0, &slot);
        if (rc) return rc;
    }
    HIP_TRY(launch_rx(a, g, h->dtype, h->LP, stream, h->rx_grid));
    return ev_end(h, slot);
}

GenArgs gen_args(ps_handle* h, int in, int out, int mx_in, int mx_out) {
    GenArgs a{};
    a.ctrl = h->ctrl;
    a.in_buf = in;
    a.out_buf = out;
    a.mx_in = mx_in;
    a.mx_out = mx_out;
    a.Xin = h->buf[in].X;
    a.Zin = h->buf[in].Z;
    a.Cin = h->buf[in].C;
    a.Xout = h->buf[out].X;
    a.Zout = h->buf[out].Z;
    a.Cout = h->buf[out].C;
    a.cap = h->cap;
    a.status = h->status;
    a.max_tiles = h->max_tiles;
    a.nq = h->nq;
    return a;
}

// The low-word arrays of binary32 general gates, allocated on first use at
// the current capacity (later capacities allocate them with the auxiliaries).
int ensure_lo(ps_handle* h) {
    if (h->has_lo) return PS_OK;
    const size_t bytes = h->cap * h->LP * sizeof(float);
    float* p[2] = {nullptr, nullptr};
    if (!grab(reinterpret_cast<void**>(&p[0]), bytes) || !grab(reinterpret_cast<void**>(&p[1]), bytes)) {
        if (p[0]) (void)hipFree(p[0]);
        return fail(PS_ERR_CAPACITY, "hipMalloc failed for the binary32 low words (%zu strings)", h->cap);
    }
    h->lo[0] = p[0];
    h->lo[1] = p[1];
    h->has_lo = true;
    return PS_OK;
}

// General gate, first half: parents and children of every string, in input
// order and in the stored x frame; tagged by sorted run when the generator
// flips few key bits.  In binary32 every output also carries the low word of
// its product (lo_live until the equal-key pass has consumed them).
int enqueue_gen_branch(ps_handle* h, int in, int out, int mx_in, double eps_in, const Stage& st) {
    GenArgs a = gen_args(h, in, out, mx_in, 1 - mx_in);
    h->lo_live = false;
    if (h->dtype == PS_F32) {
        const int rc = ensure_lo(h);
        if (rc) return rc;
        a.Lout = h->lo[out];
        h->lo_live = true;
    }
    a.eps_in = eps_in;
    a.xrot = h->xrot;
    a.xj0 = st.gen.x[0];
    a.xj1 = st.gen.x[1];
    a.zj0 = st.gen.z[0];
    a.zj1 = st.gen.z[1];
    // children form at most 2^b sorted runs (b = key bits the generator
    // flips): the output is written in the stored frame the input is sorted in
    h->gen_run_bits = -1;
    const int b = __builtin_popcountll(st.gen.x[0]) + __builtin_popcountll(st.gen.x[1]) +
                  __builtin_popcountll(st.gen.z[0]) + __builtin_popcountll(st.gen.z[1]);
    // passes: the run gather plus ceil(log2(1 + 2^b)) merge levels, against
    // the radix sort's byte digits of x and z (fewer on small registers)
    const int merge_passes = 1 + (b + 1);
    const int radix_passes = 2 * ((h->nq + 7) / 8);
    if (b <= kRunMaxBits && (b <= 4 || merge_passes < radix_passes)) {
        int q = 0;
        for (int isz = 0; isz < 2; ++isz)
            for (int bit = 0; bit < 128; ++bit) {
                const uint64_t* m = isz ? st.gen.z : st.gen.x;
                if ((m[bit >> 6] >> (bit & 63)) & 1u) {
                    // x bits sit at their stored position, bit - xrot (mod n)
                    a.run_pos[q] = static_cast<uint8_t>(isz ? bit : (bit - h->xrot + h->nq) % h->nq);
                    a.run_isz[q] = static_cast<uint8_t>(isz);
                    ++q;
                }
            }
        a.run_bits = b;
        a.Tout = h->rank[out];
        h->gen_run_bits = b;
    }
    size_t slot;
    int rc = ev_begin(h, 1, &slot);
    if (rc) return rc;
    LB_RESERVE(h, 1);
    HIP_TRY(launch_gen_branch(a, st.trig, h->dtype, h->LP, h->stream, h->grid));
    return ev_end(h, slot);
}

// General gate, second half: merge the sorted entries of buffer `in` into
// `out`, with the max of the result in slot mx_out.
int enqueue_gen_reduce(ps_handle* h, int in, int out, int mx_out) {
    GenArgs a = gen_args(h, in, out, 1 - mx_out, mx_out);
    a.Lin = h->lo_live ? h->lo[in] : nullptr;
    h->lo_live = false;
    size_t slot;
    int rc = ev_begin(h, 1, &slot);
    if (rc) return rc;
    LB_RESERVE(h, 1);
    HIP_TRY(launch_gen_reduce(a, h->dtype, h->LP, h->stream, h->grid));
    return ev_end(h, slot);
}

void drop_graphs(ps_handle* h) {
    for (auto& e : h->graph_cache) (void)hipGraphExecDestroy(e.exec);
    h->graph_cache.clear();
}

uint64_t fnv1a(uint64_t hsh, const void* p, size_t n) {
    const unsigned char* b = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) hsh = (hsh ^ b[i]) * 1099511628211ull;
    return hsh;
}

constexpr size_t kGraphCacheMax = 8;

// Enqueue the RX stages trigs[0..n) as one HIP graph: captured on the
// handle's capture stream on first use, replayed on the handle's stream when
// the same run of gates meets the same buffers, parity, pending threshold and
// capacity again.  The launches read sizes and maxima from the control block
// on the device, so a replay needs no host input.  Stage k reads buffer
// (cur + k) % 2 and uses pend0 as its pending threshold for k = 0, eps after.
int run_rx_graph(ps_handle* h, const std::vector<GateTrig>& trigs, double pend0, double eps) {
    const size_t n = trigs.size();
    uint64_t key = 1469598103934665603ull;
    const uint64_t hdr[4] = {h->alloc_gen, uint64_t(h->cap), uint64_t(h->cur | (h->mx << 1)), uint64_t(n)};
    key = fnv1a(key, hdr, sizeof hdr);
    key = fnv1a(key, &pend0, sizeof pend0);
    key = fnv1a(key, &eps, sizeof eps);
    for (const GateTrig& t : trigs) key = fnv1a(key, &t, sizeof t);
    LB_RESERVE(h, n);  // the run's look-back launches, captured or replayed
    for (const auto& e : h->graph_cache)
        if (e.key == key && e.n_stages == n) {
            HIP_TRY(hipGraphLaunch(e.exec, h->stream));
            h->graph_replays += 1;
            return PS_OK;
        }
    if (!h->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    int cur = h->cur, mx = h->mx, rc = PS_OK;
    for (size_t k = 0; k < n && rc == PS_OK; ++k) {
        rc = enqueue_rx(h, cur, 1 - cur, mx, 1 - mx, k == 0 ? pend0 : eps, trigs[k], h->cap_stream, false, true);
        cur = 1 - cur;
        mx = 1 - mx;
    }
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(h->cap_stream, &graph);
    if (rc != PS_OK || ec != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return rc != PS_OK ? rc : fail(PS_ERR_HIP, "hipStreamEndCapture: %s", hipGetErrorString(ec));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) return fail(PS_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
    if (h->graph_cache.size() >= kGraphCacheMax) {
        (void)hipGraphExecDestroy(h->graph_cache.front().exec);
        h->graph_cache.erase(h->graph_cache.begin());
    }
    h->graph_cache.push_back({key, n, exec});
    h->graph_captures += 1;
    HIP_TRY(hipGraphLaunch(exec, h->stream));
    return PS_OK;
}

// Re-sort buffer `b` (front only, with group ranks) by (rank, z).  Returns the
// buffer holding the result in *result.
// Sort of a general gate's branch output (buffer b) whose entries carry run
// tags (0 parents, 1 + class children, at most 2^bits classes): one stable
// radix pass on the tag gathers the runs, each sorted by (x, z); a tree of
// pairwise merges then sorts the whole.  Result buffer in *result.  Returns
// kUseRadix, with nothing launched, when the split buffer cannot be had.
constexpr int kUseRadix = 1;
int merge_gen_runs(ps_handle* h, int b, int bits, int* result) {
    Ctrl c;
    int rc = read_ctrl(h, &c);
    if (rc) return rc;
    const uint64_t n = c.nf[b];
    *result = b;
    if (c.err || n <= 1) return PS_OK;
    const size_t need = n / kMergeTile + kMergeMaxPairs + 2;
    if (need > h->msplit_words) {
        if (h->msplit) HIP_TRY(hipFree(h->msplit));
        h->msplit = nullptr;
        h->msplit_words = 0;
        const size_t words = need + need / 4;
        if (hipMalloc(reinterpret_cast<void**>(&h->msplit), words * 8) != hipSuccess) {
            (void)hipGetLastError();
            return kUseRadix;  // the radix sort needs no memory of its own
        }
        h->msplit_words = words;
    }
    SortPlan plan{};
    plan.npass = 1;
    plan.lo[0] = 128;  // the tag sits in the rank word of the key
    plan.w[0] = static_cast<uint8_t>(bits + 1);
    const int nrun = 1 + (1 << bits);
    HIP_TRY(hipMemsetAsync(h->hist, 0, 256 * sizeof(uint32_t), h->stream));
    HIP_TRY(launch_sort_hist(h->ctrl, b, h->rank[b], h->buf[b].Z, h->buf[b].X, plan, h->hist, h->stream, h->grid));
    std::vector<uint32_t> cnt(256);
    HIP_TRY(hipMemcpyAsync(cnt.data(), h->hist, 256 * sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    std::vector<uint32_t> base(256, 0);
    std::vector<std::pair<uint64_t, uint64_t>> segs;  // (start, length) of the non-empty runs
    uint64_t run = 0;
    for (int k = 0; k < 256; ++k) {
        base[k] = static_cast<uint32_t>(run);
        if (cnt[k] && k >= nrun) return fail(PS_ERR_DEVICE, "run tag %d out of range", k);
        if (cnt[k]) segs.push_back({run, cnt[k]});
        run += cnt[k];
    }
    if (run != n) return fail(PS_ERR_DEVICE, "run tags cover %llu of %llu entries", (unsigned long long)run,
                              (unsigned long long)n);
    if (segs.size() <= 1) return PS_OK;  // a single run: sorted already
    HIP_TRY(hipMemcpyAsync(h->digit_base, base.data(), 256 * sizeof(uint32_t), hipMemcpyHostToDevice, h->stream));
    SortPassArgs a{};
    a.ctrl = h->ctrl;
    a.n = n;
    a.lo = 128;
    a.w = bits + 1;
    a.digit_base = h->digit_base;
    a.Rs = h->rank[b];
    a.Zs = h->buf[b].Z;
    a.Xs = h->buf[b].X;
    a.Cs = h->buf[b].C;
    a.Rd = h->rank[1 - b];
    a.Zd = h->buf[1 - b].Z;
    a.Xd = h->buf[1 - b].X;
    a.Cd = h->buf[1 - b].C;
    a.status = h->status;
    a.max_tiles = h->status_words / 256;
    a.dst_buf = 1 - b;
    if (h->lo_live) {
        a.Ls = h->lo[b];
        a.Ld = h->lo[1 - b];
    }
    size_t slot;
    rc = ev_begin(h, 2, &slot);
    if (rc) return rc;
    LB_RESERVE(h, 1);
    HIP_TRY(launch_sort_pass(a, 8, h->dtype, h->LP, h->stream, h->grid));
    rc = ev_end(h, slot);
    if (rc) return rc;
    h->sort_passes += 1;
    h->sort_elems += double(n);
    int src = 1 - b;
    while (segs.size() > 1) {
        MergeArgs m{};
        m.ctrl = h->ctrl;
        m.n = n;
        m.dst_buf = 1 - src;
        std::vector<std::pair<uint64_t, uint64_t>> next;
        uint64_t tiles = 0;
        for (size_t i = 0; i < segs.size(); i += 2) {
            MergePair& P = m.pairs[m.npairs++];
            P.a0 = segs[i].first;
            P.na = segs[i].second;
            P.nb = i + 1 < segs.size() ? segs[i + 1].second : 0;
            P.tile0 = tiles;
            tiles += (P.na + P.nb + kMergeTile - 1) / kMergeTile;
            next.push_back({P.a0, P.na + P.nb});
        }
        m.ntiles = tiles;
        m.Xs = h->buf[src].X;
        m.Zs = h->buf[src].Z;
        m.Cs = h->buf[src].C;
        m.Xd = h->buf[1 - src].X;
        m.Zd = h->buf[1 - src].Z;
        m.Cd = h->buf[1 - src].C;
        m.split = h->msplit;
        if (h->lo_live) {
            m.Ls = h->lo[src];
            m.Ld = h->lo[1 - src];
        }
        rc = ev_begin(h, 2, &slot);
        if (rc) return rc;
        HIP_TRY(launch_merge_pairs(m, h->dtype, h->LP, h->stream));
        rc = ev_end(h, slot);
        if (rc) return rc;
        h->sort_passes += 1;
        h->sort_elems += double(n);
        segs.swap(next);
        src = 1 - src;
    }
    h->run_merges += 1;
    *result = src;
    HIP_TRY(hipStreamSynchronize(h->stream));
    return ev_collect(h);
}

// Radix-sort candidates: (digit bits, items per thread).  Narrower digits
// give longer runs per bucket in each tile (better write coalescing) at the
// price of more passes; larger tiles do the same for fewer look-back steps.
constexpr int kSortCands = 6;
constexpr int kSortCandBits[kSortCands] = {8, 8, 7, 6, 7, 6};
constexpr int kSortCandIpt[kSortCands] = {8, 16, 16, 16, 8, 8};
constexpr uint64_t kSortTuneMin = 1u << 16;  // smaller sorts use candidate 0 untimed

SortPlan make_sort_plan(int nq, bool full_key, int rbits, int bits) {
    SortPlan p{};
    auto seg = [&](int base, int len) {
        for (int o = 0; o < len; o += bits) {
            p.lo[p.npass] = static_cast<uint16_t>(base + o);
            p.w[p.npass] = static_cast<uint8_t>(std::min(bits, len - o));
            ++p.npass;
        }
    };
    seg(0, nq);                          // z, least significant
    if (full_key) seg(192, nq);          // then x
    else seg(128, rbits);                // or the x-group rank
    return p;
}

int pick_sort_candidate(const ps_handle* h, int kind, int cls, uint64_t n) {
    if (h->sort_force >= 0) return h->sort_force;
    if (n < kSortTuneMin) return 0;
    const float* t = h->sort_ns[kind][cls];
    int best = 0;
    for (int c = 0; c < kSortCands; ++c) {
        if (t[c] == 0.0f) return c;  // not tried in this class yet
        if (t[c] < t[best]) best = c;
    }
    return best;
}

int sort_by_rank_z(ps_handle* h, int b, int* result, bool full_key = false, bool try_groups = true,
                   bool* overflowed = nullptr, int run_bits = -1, bool xor_groups = false) {
    if (overflowed) *overflowed = false;
    Ctrl c;
    int rc = read_ctrl(h, &c);
    if (rc) return rc;
    if (c.err) return PS_OK;  // a failed stage before: nothing to sort
    const uint64_t n = c.nf[b];
    *result = b;
    if (n <= 1) return PS_OK;
    if (try_groups) {  // every x-group small enough: one pass sorts each group inside a workgroup
        GroupSortArgs g{};
        g.ctrl = h->ctrl;
        g.in_buf = b;
        g.out_buf = 1 - b;
        g.Xs = h->buf[b].X;
        g.Zs = h->buf[b].Z;
        g.Cs = h->buf[b].C;
        g.Xd = h->buf[1 - b].X;
        g.Zd = h->buf[1 - b].Z;
        g.Cd = h->buf[1 - b].C;
        if (h->lo_live) {
            g.Ls = h->lo[b];
            g.Ld = h->lo[1 - b];
        }
        g.xor_order = xor_groups ? 1 : 0;
        size_t slot;
        rc = ev_begin(h, 2, &slot);
        if (rc) return rc;
        HIP_TRY(launch_group_sort(g, h->dtype, h->LP, h->stream, xor_groups ? h->grid : h->grid / 2));
        rc = ev_end(h, slot);
        if (rc) return rc;
        Ctrl c2;
        rc = read_ctrl(h, &c2);
        if (rc) return rc;
        h->sort_passes += 1;
        h->sort_elems += double(n);
        if (c2.aux[2] == 0) {
            *result = 1 - b;
            return PS_OK;
        }
        // a group too large for one workgroup: radix sort from the untouched input
        if (overflowed) *overflowed = true;
        const uint64_t zero = 0;
        HIP_TRY(hipMemcpyAsync(&h->ctrl->aux[2], &zero, 8, hipMemcpyHostToDevice, h->stream));
        HIP_TRY(hipMemcpyAsync(&h->ctrl->nf[1 - b], &zero, 8, hipMemcpyHostToDevice, h->stream));
    }
    if (full_key && run_bits >= 0) {
        rc = merge_gen_runs(h, b, run_bits, result);
        if (rc != kUseRadix) return rc;
        *result = b;
    }
    const int kind = full_key ? 1 : 0;
    int cls = 0;
    while (cls < 63 && (uint64_t(2) << cls) <= n) ++cls;
    const int cand = pick_sort_candidate(h, kind, cls, n);
    const int bits = kSortCandBits[cand], ipt = kSortCandIpt[cand];
    int rbits = 32;
    if (!full_key && c.nranks > 0 && c.nranks <= (uint64_t(1) << 32)) {
        rbits = 1;
        while (rbits < 32 && (uint64_t(1) << rbits) < c.nranks) ++rbits;
    }
    const SortPlan plan = make_sort_plan(h->nq, full_key, rbits, bits);
    HIP_TRY(hipMemsetAsync(h->hist, 0, kSortMaxPasses * 256 * sizeof(uint32_t), h->stream));
    HIP_TRY(launch_sort_hist(h->ctrl, b, full_key ? nullptr : h->rank[b], h->buf[b].Z, h->buf[b].X, plan, h->hist,
                             h->stream, h->grid));
    std::vector<uint32_t> hist(plan.npass * 256);
    HIP_TRY(hipMemcpyAsync(hist.data(), h->hist, hist.size() * sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    std::vector<int> passes;  // plan entries whose digit is not constant
    for (int p = 0; p < plan.npass; ++p) {
        int nonzero = 0;
        for (int k = 0; k < 256; ++k) nonzero += hist[p * 256 + k] != 0;
        if (nonzero > 1) passes.push_back(p);
    }
    if (passes.empty()) return PS_OK;
    std::vector<uint32_t> bases(passes.size() * 256);
    for (size_t i = 0; i < passes.size(); ++i) {
        uint64_t run = 0;
        for (int k = 0; k < 256; ++k) {
            bases[i * 256 + k] = static_cast<uint32_t>(run);
            run += hist[passes[i] * 256 + k];
        }
    }
    HIP_TRY(hipMemcpyAsync(h->digit_base, bases.data(), bases.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                           h->stream));
    const bool tune = h->sort_force < 0 && n >= kSortTuneMin;
    if (tune && !h->sort_ev[0]) {
        HIP_TRY(hipEventCreateWithFlags(&h->sort_ev[0], hipEventDisableSystemFence));
        HIP_TRY(hipEventCreateWithFlags(&h->sort_ev[1], hipEventDisableSystemFence));
    }
    if (tune) HIP_TRY(hipEventRecord(h->sort_ev[0], h->stream));
    int src = b;
    for (size_t i = 0; i < passes.size(); ++i) {
        const int dst = 1 - src;
        SortPassArgs a{};
        a.ctrl = h->ctrl;
        a.n = n;
        a.lo = plan.lo[passes[i]];
        a.w = plan.w[passes[i]];
        a.digit_base = h->digit_base + i * 256;
        a.Rs = full_key ? nullptr : h->rank[src];
        a.Zs = h->buf[src].Z;
        a.Xs = h->buf[src].X;
        a.Cs = h->buf[src].C;
        a.Rd = full_key ? nullptr : h->rank[dst];
        a.Zd = h->buf[dst].Z;
        a.Xd = h->buf[dst].X;
        a.Cd = h->buf[dst].C;
        a.status = h->status;
        a.max_tiles = h->status_words / 256;
        a.dst_buf = dst;
        if (h->lo_live) {
            a.Ls = h->lo[src];
            a.Ld = h->lo[dst];
        }
        size_t slot;
        rc = ev_begin(h, 2, &slot);
        if (rc) return rc;
        LB_RESERVE(h, 1);
        HIP_TRY(launch_sort_pass(a, ipt, h->dtype, h->LP, h->stream, h->grid));
        rc = ev_end(h, slot);
        if (rc) return rc;
        h->sort_passes += 1;
        h->sort_elems += double(n);
        src = dst;
    }
    if (tune) HIP_TRY(hipEventRecord(h->sort_ev[1], h->stream));
    *result = src;
    // keep the host copy of the digit bases alive until the copy has run
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->radix_sorts += 1;
    h->sort_last = cand;
    if (tune) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, h->sort_ev[0], h->sort_ev[1]));
        const float ns = std::max(1e-6f, ms * 1e6f / float(n));
        float& slot = h->sort_ns[kind][cls][cand];
        slot = (slot == 0.0f) ? ns : std::min(slot, ns);
    }
    return ev_collect(h);
}

int validate_key(int nq, const ps_pauli& p) {
    for (int w = 0; w < 2; ++w) {
        const int lo = w * 64;
        if (nq >= lo + 64) continue;
        const uint64_t allowed = (nq <= lo) ? 0ull : ((1ull << (nq - lo)) - 1ull);
        if ((p.x[w] & ~allowed) || (p.z[w] & ~allowed)) return 0;
    }
    return 1;
}

// Apply the pending truncation (if any) so the state is exact as stored.
int materialize(ps_handle* h) {
    if (!(h->pend > 0.0)) return PS_OK;
    const int out = 1 - h->cur, mx_out = 1 - h->mx;
    int rc = enqueue_compact(h, h->cur, out, h->mx, mx_out, h->pend, nullptr, 0, false);
    if (rc) return rc;
    h->cur = out;
    h->mx = mx_out;
    h->pend = -1.0;
    return check_no_error(h, "truncation");
}

// ---------------------------------------------------------------- histogram
int check_histogram_args(ps_handle* h, int lane, const double* edges, int n_bins, uint64_t* counts) {
    if (!h || !edges || !counts) return fail(PS_ERR_INVALID, "NULL argument");
    if (h->broken) return fail(PS_ERR_DEVICE, "handle is no longer usable");
    if (lane < 0 || lane >= h->L) return fail(PS_ERR_INVALID, "lane %d out of range", lane);
    if (n_bins < 1 || n_bins > kHistMaxBins) return fail(PS_ERR_INVALID, "n_bins must be in 1..%d", kHistMaxBins);
    for (int k = 0; k <= n_bins; ++k) {
        if (!std::isfinite(edges[k])) return fail(PS_ERR_NONFINITE, "edge %d is not finite", k);
        if (k > 0 && !(edges[k] > edges[k - 1])) return fail(PS_ERR_INVALID, "edges must increase");
    }
    return PS_OK;
}

// Counts of the current operator into host counts[n_bins + 2], with device
// memory dE (n_bins + 1 doubles) and dC (n_bins + 2 words) supplied by the
// caller.  A pending truncation is applied inside the counting kernel.
int run_histogram(ps_handle* h, int lane, const double* edges, int n_bins, int is_signed, uint64_t* counts,
                  double* dE, uint64_t* dC) {
    HistArgs a{};
    a.ctrl = h->ctrl;
    a.buf = h->cur;
    a.mx = h->mx;
    a.C = h->buf[h->cur].C;
    a.cap = h->cap;
    a.lane = lane;
    a.nbins = n_bins;
    a.is_signed = is_signed ? 1 : 0;
    a.eps_pend = h->pend;
    a.edges = dE;
    a.counts = dC;
    hipError_t e = hipMemcpyAsync(dE, edges, size_t(n_bins + 1) * 8, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = launch_fill_u64(dC, 0, size_t(n_bins + 2), h->stream);
    if (e == hipSuccess) e = launch_histogram(a, h->dtype, h->LP, h->stream, h->grid);
    if (e == hipSuccess) e = hipMemcpyAsync(counts, dC, size_t(n_bins + 2) * 8, hipMemcpyDeviceToHost, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return fail(PS_ERR_HIP, "histogram: %s", hipGetErrorString(e));
    return PS_OK;
}

// ---------------------------------------------------------------- fixed scratch
// Device memory of pauli_sum_histogram_noalloc: the bin edges (kHistMaxBins + 1
// doubles) followed by the counters (kHistMaxBins + 2 words), 64 KiB and a bit
// in one fixed array.  Every GPU the library runs on holds its own copy until
// the process ends.  In host code `scratch` names a host-side stand-in, not
// device memory: its device address is looked up once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// handed to kernels and copies.
constexpr size_t kScratchCountsAt = kHistMaxBins + 1;
constexpr size_t kScratchWords = kScratchCountsAt + kHistMaxBins + 2;
static __device__ __align__(256) uint64_t scratch[kScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on device dev, which must be current.
int scratch_address(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(PS_ERR_UNSUPPORTED, "device %d beyond the scratch table", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(PS_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PS_OK;
}

}  // namespace

// ================================================================ C ABI

extern "C" {

const char* ps_last_error(void) { return g_last_error.c_str(); }

int pauli_sum_create(int n_qubits, int n_lanes, int dtype, size_t capacity, const ps_pauli* terms,
                     const double* coeffs, size_t n_terms, void* hip_stream, ps_handle** out) {
    if (!out) return fail(PS_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (n_qubits < 1 || n_qubits > 128) return fail(PS_ERR_INVALID, "n_qubits must be in 1..128");
    if (n_lanes < 1 || n_lanes > kMaxLanes) return fail(PS_ERR_INVALID, "n_lanes must be in 1..32");
    if (dtype != PS_F64 && dtype != PS_F32) return fail(PS_ERR_INVALID, "dtype must be PS_F64 or PS_F32");
    if (n_terms && (!terms || !coeffs)) return fail(PS_ERR_INVALID, "terms/coeffs NULL");
    for (size_t t = 0; t < n_terms; ++t) {
        if (!validate_key(n_qubits, terms[t]))
            return fail(PS_ERR_INVALID, "term %zu has bits at or above n_qubits=%d", t, n_qubits);
        for (int a = 0; a < n_lanes; ++a)
            if (!std::isfinite(coeffs[t * n_lanes + a]))
                return fail(PS_ERR_NONFINITE, "coefficient %zu lane %d is not finite", t, a);
    }
    int dev_count = 0;
    const hipError_t de = hipGetDeviceCount(&dev_count);
    if (de != hipSuccess || dev_count < 1)
        return fail(PS_ERR_HIP, "no HIP device available (%s)", hipGetErrorString(de));

    ps_handle* h = new ps_handle;
    h->nq = n_qubits;
    h->L = n_lanes;
    h->LP = lanes_pad(n_lanes);
    h->dtype = dtype;
    h->csize = size_t(h->LP) * (dtype == PS_F64 ? 8 : 4);
    h->stream = static_cast<hipStream_t>(hip_stream);
    {
        int dev = 0, cus = 0;
        (void)hipGetDevice(&dev);
        h->dev = dev;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            h->grid = cus * 4;
        const int per_cu = rx_blocks_per_cu(dtype, h->LP);
        h->rx_grid = (cus > 0 && per_cu > 0) ? std::min(h->grid, cus * per_cu) : h->grid;
    }

    // host-side canonical order: (stored x, z) ascending, duplicates summed
    struct Row {
        U128 x, z;
        size_t src;
    };
    std::vector<Row> rows(n_terms);
    for (size_t t = 0; t < n_terms; ++t)
        rows[t] = {{terms[t].x[0], terms[t].x[1]}, {terms[t].z[0], terms[t].z[1]}, t};
    auto less = [](const Row& a, const Row& b) {
        if (a.x.hi != b.x.hi) return a.x.hi < b.x.hi;
        if (a.x.lo != b.x.lo) return a.x.lo < b.x.lo;
        if (a.z.hi != b.z.hi) return a.z.hi < b.z.hi;
        return a.z.lo < b.z.lo;
    };
    std::stable_sort(rows.begin(), rows.end(), less);
    std::vector<ulonglong2> hx, hz;
    std::vector<double> hc;
    for (size_t i = 0; i < rows.size(); ++i) {
        const Row& r = rows[i];
        if (!hx.empty() && hx.back().x == r.x.lo && hx.back().y == r.x.hi && hz.back().x == r.z.lo &&
            hz.back().y == r.z.hi) {
            for (int a = 0; a < n_lanes; ++a) hc[(hx.size() - 1) * h->LP + a] += coeffs[r.src * n_lanes + a];
            continue;
        }
        hx.push_back(make_ulonglong2(r.x.lo, r.x.hi));
        hz.push_back(make_ulonglong2(r.z.lo, r.z.hi));
        for (int a = 0; a < h->LP; ++a) hc.push_back(a < n_lanes ? coeffs[r.src * n_lanes + a] : 0.0);
    }
    const size_t n = hx.size();
    size_t cap = std::max<size_t>({capacity, n + 1024, size_t(1) << 16});
    h->cap = cap;
    int rc = PS_OK;
    auto bail = [&](int code) {
        free_buffers(h);
        if (h->ctrl) (void)hipFree(h->ctrl);
        if (h->hist) (void)hipFree(h->hist);
        if (h->digit_base) (void)hipFree(h->digit_base);
        if (h->partial) (void)hipFree(h->partial);
        if (h->red_out) (void)hipFree(h->red_out);
        if (h->cgens) (void)hipFree(h->cgens);
        delete h;
        return code;
    };
    if (hipMalloc(reinterpret_cast<void**>(&h->ctrl), sizeof(Ctrl)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&h->hist), kSortMaxPasses * 256 * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&h->digit_base), kSortMaxPasses * 256 * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&h->partial), 2 * kReduceBlocks * kMaxLanes * sizeof(double)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&h->red_out), kMaxLanes * sizeof(double)) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&h->cgens),
                  kMaxCliffGens * sizeof(CliffGen) + kMaxCliffGroups * sizeof(CliffGroup)) != hipSuccess) {
        (void)hipGetLastError();
        return bail(fail(PS_ERR_CAPACITY, "hipMalloc failed for handle scratch"));
    }
    rc = alloc_buffers(h, cap);
    if (rc) return bail(rc);
    Ctrl c;
    std::memset(&c, 0, sizeof c);
    c.epoch = 1;
    c.nf[0] = n;
    std::vector<double> mx(kMaxLanes, 0.0);
    for (size_t i = 0; i < n; ++i)
        for (int a = 0; a < n_lanes; ++a) mx[a] = std::fmax(mx[a], std::fabs(hc[i * h->LP + a]));
    for (int a = 0; a < n_lanes; ++a) std::memcpy(&c.maxbits[0][a], &mx[a], 8);
    if (hipMemcpyAsync(h->ctrl, &c, sizeof c, hipMemcpyHostToDevice, h->stream) != hipSuccess)
        return bail(fail(PS_ERR_HIP, "upload ctrl"));
    if (n) {
        if (hipMemcpyAsync(h->buf[0].X, hx.data(), n * sizeof(ulonglong2), hipMemcpyHostToDevice, h->stream) !=
                hipSuccess ||
            hipMemcpyAsync(h->buf[0].Z, hz.data(), n * sizeof(ulonglong2), hipMemcpyHostToDevice, h->stream) !=
                hipSuccess)
            return bail(fail(PS_ERR_HIP, "upload keys"));
        if (dtype == PS_F64) {
            if (hipMemcpyAsync(h->buf[0].C, hc.data(), n * h->LP * 8, hipMemcpyHostToDevice, h->stream) != hipSuccess)
                return bail(fail(PS_ERR_HIP, "upload coefficients"));
            if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(fail(PS_ERR_HIP, "sync"));
        } else {
            std::vector<float> f(hc.size());
            for (size_t i = 0; i < hc.size(); ++i) f[i] = static_cast<float>(hc[i]);
            if (hipMemcpyAsync(h->buf[0].C, f.data(), f.size() * 4, hipMemcpyHostToDevice, h->stream) != hipSuccess)
                return bail(fail(PS_ERR_HIP, "upload coefficients"));
            if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(fail(PS_ERR_HIP, "sync"));
        }
    }
    if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(fail(PS_ERR_HIP, "sync"));
    h->n_host = n;
    *out = h;
    return PS_OK;
}

int pauli_sum_destroy(ps_handle* h) {
    if (!h) return PS_OK;
    (void)hipStreamSynchronize(h->stream);
    free_buffers(h);
    if (h->ctrl) (void)hipFree(h->ctrl);
    if (h->hist) (void)hipFree(h->hist);
    if (h->digit_base) (void)hipFree(h->digit_base);
    if (h->partial) (void)hipFree(h->partial);
    if (h->red_out) (void)hipFree(h->red_out);
    if (h->cgens) (void)hipFree(h->cgens);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    for (hipEvent_t e : h->sort_ev)
        if (e) (void)hipEventDestroy(e);
    if (h->msplit) (void)hipFree(h->msplit);
    if (h->has_scorer) scorer_free(&h->scorer);
    drop_graphs(h);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    delete h;
    return PS_OK;
}

int pauli_sum_gates_applied(ps_handle* h, size_t* n) {
    if (!h || !n) return fail(PS_ERR_INVALID, "NULL argument");
    *n = h->gates_applied;
    return PS_OK;
}

int apply_rotation_layer(ps_handle* h, const ps_pauli* gens, const double* thetas, size_t n_gates, double rel_eps,
                         int trunc_mode) {
    if (!h) return fail(PS_ERR_INVALID, "handle is NULL");
    if (h->broken) return fail(PS_ERR_DEVICE, "handle is no longer usable after a device failure");
    h->gates_applied = 0;
    h->lo_live = false;
    if (n_gates == 0) return PS_OK;
    if (!gens || !thetas) return fail(PS_ERR_INVALID, "gens/thetas NULL");
    if (trunc_mode != PS_TRUNC_NONE && trunc_mode != PS_TRUNC_MAGNITUDE && trunc_mode != PS_TRUNC_LEARNED)
        return fail(PS_ERR_INVALID, "unknown trunc_mode %d", trunc_mode);
    if (trunc_mode == PS_TRUNC_LEARNED && !h->has_scorer)
        return fail(PS_ERR_INVALID, "PS_TRUNC_LEARNED needs pauli_sum_load_scorer first");
    if (std::isnan(rel_eps)) return fail(PS_ERR_NONFINITE, "rel_eps is NaN");
    const double eps_learned = (trunc_mode == PS_TRUNC_LEARNED && rel_eps > 0.0) ? rel_eps * h->learned_ratio : -1.0;
    const double eps = (trunc_mode == PS_TRUNC_NONE || !(rel_eps > 0.0)) ? -1.0 : rel_eps;
    for (size_t g = 0; g < n_gates; ++g) {
        if (!validate_key(h->nq, gens[g])) return fail(PS_ERR_INVALID, "generator %zu has bits above n_qubits", g);
        for (int a = 0; a < h->L; ++a)
            if (!std::isfinite(thetas[g * h->L + a])) return fail(PS_ERR_NONFINITE, "theta %zu lane %d", g, a);
    }

    // ---- plan: runs of Z-only Clifford gates, and sigma_x rotations on the
    // qubit at stored bit 0.
    std::vector<Stage> stages;
    int xrot = h->xrot;
    for (size_t g = 0; g < n_gates;) {
        const ps_pauli& G = gens[g];
        double cs[kMaxLanes], sn[kMaxLanes];
        int kk[kMaxLanes];
        bool same_k = true;
        for (int a = 0; a < h->L; ++a) {
            kk[a] = classify(thetas[g * h->L + a], &cs[a], &sn[a]);
            if (kk[a] != kk[0]) same_k = false;
        }
        const bool zonly = (G.x[0] | G.x[1]) == 0;
        const bool zero = zonly && (G.z[0] | G.z[1]) == 0;
        if (zero) {  // identity generator: the gate is a global phase
            Stage s{};
            s.kind = ST_CLIFF;
            s.gate_first = g;
            s.gate_count = 1;
            s.needs_sort = false;
            stages.push_back(s);
            ++g;
            continue;
        }
        if (zonly && same_k && kk[0] >= 0) {
            Stage s{};
            s.kind = ST_CLIFF;
            s.gate_first = g;
            s.needs_sort = false;
            size_t e = g;
            while (e < n_gates && s.gens.size() < size_t(kMaxCliffGens)) {
                const ps_pauli& E = gens[e];
                if ((E.x[0] | E.x[1]) != 0) break;
                double c2[kMaxLanes], s2[kMaxLanes];
                int k0 = -2;
                bool ok = true;
                for (int a = 0; a < h->L; ++a) {
                    const int k = classify(thetas[e * h->L + a], &c2[a], &s2[a]);
                    if (a == 0) k0 = k;
                    if (k != k0) ok = false;
                }
                if (!ok || k0 < 0) break;
                if (k0 != 0 && (E.z[0] | E.z[1]) != 0) {
                    CliffGen cg{};
                    cg.z0 = E.z[0];
                    cg.z1 = E.z[1];
                    cg.kodd = (k0 & 1) ? 1u : 0u;
                    cg.neg = (k0 == 3 || k0 == 2) ? 1u : 0u;
                    s.gens.push_back(cg);
                    if (cg.kodd) s.needs_sort = true;
                }
                ++e;
            }
            s.gate_count = e - g;
            stages.push_back(std::move(s));
            g = e;
            continue;
        }
        // sigma_x on one qubit?
        const bool single_x = (G.z[0] | G.z[1]) == 0 && (__builtin_popcountll(G.x[0]) + __builtin_popcountll(G.x[1])) == 1;
        if (single_x) {
            const int q = G.x[0] ? __builtin_ctzll(G.x[0]) : 64 + __builtin_ctzll(G.x[1]);
            if (q == xrot % h->nq) {
                Stage s{};
                s.kind = ST_RX;
                s.gate_first = g;
                s.gate_count = 1;
                s.qubit = q;
                GateTrig& t = s.trig;
                std::memset(&t, 0, sizeof t);
                bool any_c = false, any_s = false;
                for (int a = 0; a < h->L; ++a) {
                    t.cs[a] = cs[a];
                    t.sn[a] = sn[a];
                    split_f32(cs[a], &t.cs_hi[a], &t.cs_lo[a]);
                    split_f32(sn[a], &t.sn_hi[a], &t.sn_lo[a]);
                    any_c |= cs[a] != 0.0;
                    any_s |= sn[a] != 0.0;
                }
                t.any_c = any_c;
                t.any_s = any_s;
                t.zword = q >> 6;
                t.zbit = q & 63;
                stages.push_back(s);
                xrot = (xrot + 1) % h->nq;
                ++g;
                continue;
            }
        }
        {  // any other Pauli rotation: branch, full sort, merge
            Stage s{};
            s.kind = ST_GEN;
            s.gate_first = g;
            s.gate_count = 1;
            s.gen = G;
            GateTrig& t = s.trig;
            std::memset(&t, 0, sizeof t);
            bool any_c = false, any_s = false;
            for (int a = 0; a < h->L; ++a) {
                t.cs[a] = cs[a];
                t.sn[a] = sn[a];
                split_f32(cs[a], &t.cs_hi[a], &t.cs_lo[a]);
                split_f32(sn[a], &t.sn_hi[a], &t.sn_lo[a]);
                any_c |= cs[a] != 0.0;
                any_s |= sn[a] != 0.0;
            }
            t.any_c = any_c;
            t.any_s = any_s;
            stages.push_back(s);
            ++g;
        }
    }

    // ---- execute.  Stages are enqueued back to back; the host synchronises
    // after a Clifford stage that needs a re-sort and at the end.  A stage
    // that runs out of capacity raises kErrCapacity, every later kernel turns
    // into a no-op, and the stage's input buffer is intact: grow and resume.
    Ctrl c0;
    int rc = read_ctrl(h, &c0);
    if (rc) return rc;
    if (c0.err) return fail(PS_ERR_DEVICE, "device error bits 0x%x before the layer", c0.err);
    const uint64_t zero64 = 0;
    HIP_TRY(hipMemcpyAsync(&h->ctrl->stages_done, &zero64, 8, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));

    struct Launched {
        size_t stage;
        int cur, mx, xrot;
        double pend;
    };
    size_t si = 0;
    while (si < stages.size()) {
        std::vector<Launched> launched;
        bool sort_after = false, gen_after = false, gen_zonly = false;
        for (; si < stages.size(); ++si) {
            Stage& s = stages[si];
            const bool noop = s.kind == ST_CLIFF && s.gens.empty() && !(h->pend > 0.0) && !(eps_learned > 0.0);
            if (noop) {
                // the gates leave every magnitude (and the max) unchanged:
                // only the pending threshold of this layer is recorded
                if (eps > 0.0) h->pend = std::max(h->pend, eps);
                continue;
            }
            if (s.kind == ST_RX && h->graphs && !h->timing) {
                size_t j = si;
                std::vector<GateTrig> trigs;
                while (j < stages.size() && stages[j].kind == ST_RX) trigs.push_back(stages[j++].trig);
                rc = run_rx_graph(h, trigs, h->pend, eps);
                if (rc) return rc;
                for (size_t k = si; k < j; ++k) {
                    launched.push_back({k, h->cur, h->mx, h->xrot, h->pend});
                    h->xrot = (h->xrot + 1) % h->nq;
                    h->cur = 1 - h->cur;
                    h->mx = 1 - h->mx;
                    h->pend = eps;
                }
                si = j - 1;  // the loop increment moves past the run
                continue;
            }
            launched.push_back({si, h->cur, h->mx, h->xrot, h->pend});
            const int in = h->cur, out = 1 - h->cur, mx_in = h->mx, mx_out = 1 - h->mx;
            if (s.kind == ST_GEN) {  // branch now; sort and merge after the synchronisation
                rc = enqueue_gen_branch(h, in, out, mx_in, h->pend, s);
                if (rc) return rc;
                h->cur = out;
                gen_zonly = (s.gen.x[0] | s.gen.x[1]) == 0;  // outputs keep the stored frame
                h->pend = -1.0;
                gen_after = true;
                ++si;
                break;
            }
            if (s.kind == ST_RX) {
                rc = enqueue_rx(h, in, out, mx_in, mx_out, h->pend, s.trig);
                if (rc) return rc;
                h->xrot = (h->xrot + 1) % h->nq;
            } else {
                std::vector<CliffGroup> groups;
                std::vector<CliffGen> rest;
                group_cliff_gens(s.gens, groups, rest);
                CliffGroup* dgroups = reinterpret_cast<CliffGroup*>(h->cgens + kMaxCliffGens);
                if (!rest.empty())
                    HIP_TRY(hipMemcpyAsync(h->cgens, rest.data(), rest.size() * sizeof(CliffGen),
                                           hipMemcpyHostToDevice, h->stream));
                if (!groups.empty())
                    HIP_TRY(hipMemcpyAsync(dgroups, groups.data(), groups.size() * sizeof(CliffGroup),
                                           hipMemcpyHostToDevice, h->stream));
                bool neg_is_k = true;  // e.g. every generator at theta = -pi/2
                for (const CliffGroup& c : groups) neg_is_k = neg_is_k && c.k0 == c.n0 && c.k1 == c.n1;
                rc = enqueue_compact(h, in, out, mx_in, mx_out, h->pend, h->cgens, int(rest.size()),
                                     s.needs_sort, int(s.gate_count), eps_learned, dgroups, int(groups.size()),
                                     neg_is_k);
                if (rc) return rc;
                if (!s.gens.empty()) HIP_TRY(hipStreamSynchronize(h->stream));  // cgens reused by the next run
            }
            h->cur = out;
            h->mx = mx_out;
            h->pend = eps;
            if (s.kind == ST_CLIFF && s.needs_sort) {
                sort_after = true;
                ++si;
                break;
            }
        }
        Ctrl c;
        rc = read_ctrl(h, &c);
        if (rc) return rc;
        if (c.err & kErrLookback) {
            h->broken = true;
            return fail(PS_ERR_DEVICE, "look-back wait timed out (handle is no longer usable)");
        }
        if (c.err & kErrCapacity) {
            if (c.stages_done >= launched.size())
                return fail(PS_ERR_DEVICE, "capacity error with no failing stage");
            const Launched& L = launched[c.stages_done];
            h->cur = L.cur;
            h->mx = L.mx;
            h->xrot = L.xrot;
            h->pend = L.pend;
            const int grc = grow(h, h->cur, c.need);
            rc = clear_error(h, 1 - h->mx);
            HIP_TRY(hipMemcpyAsync(&h->ctrl->stages_done, &zero64, 8, hipMemcpyHostToDevice, h->stream));
            HIP_TRY(hipStreamSynchronize(h->stream));
            if (grc) {
                h->gates_applied = stages[L.stage].gate_first;
                return grc;
            }
            if (rc) return rc;
            si = L.stage;
            continue;
        }
        if (c.err) return fail(PS_ERR_DEVICE, "kernel error bits 0x%x", c.err);
        HIP_TRY(hipMemcpyAsync(&h->ctrl->stages_done, &zero64, 8, hipMemcpyHostToDevice, h->stream));
        h->n_host = c.nf[h->cur] + c.nb[h->cur];
        if (sort_after) {
            int res = h->cur;
            // after a Clifford run: each x-group is its sorted run XORed with one mask
            rc = sort_by_rank_z(h, h->cur, &res, false, true, nullptr, -1, true);
            if (rc) return rc;
            h->cur = res;
            rc = check_no_error(h, "re-sort");
            if (rc) return rc;
        }
        if (gen_after) {  // general gate: sort the branch output by (x, z), merge equal keys
            const int mx_branch = h->mx;  // zeroed by the branch; the merge's max goes to the other slot
            int res = h->cur;
            // x_J = 0: outputs stay in their x-groups, which keep their order:
            // sort inside the groups; otherwise the full (x, z) radix sort
            const bool try_groups = gen_zonly && h->gs_skip == 0;
            if (gen_zonly && h->gs_skip > 0) --h->gs_skip;
            bool over = false;
            rc = sort_by_rank_z(h, h->cur, &res, true, try_groups, &over, h->gen_run_bits);
            if (over) h->gs_skip = 32;
            if (rc) return rc;
            rc = enqueue_gen_reduce(h, res, 1 - res, 1 - mx_branch);
            if (rc) return rc;
            h->cur = 1 - res;
            h->mx = 1 - mx_branch;
            h->pend = eps;
            Ctrl cg;
            rc = read_ctrl(h, &cg);
            if (rc) return rc;
            if (cg.err) return fail(PS_ERR_DEVICE, "general gate: kernel error bits 0x%x", cg.err);
            h->n_host = cg.nf[h->cur] + cg.nb[h->cur];
        }
        h->gates_applied = (si < stages.size()) ? stages[si].gate_first : n_gates;
        // grow ahead of a layer when the operator is close to the capacity
        if (si < stages.size() && h->n_host + h->n_host / 3 + 1024 > h->cap) {
            rc = grow(h, h->cur, h->n_host + h->n_host / 3 + 1024);
            if (rc && rc != PS_ERR_CAPACITY) return rc;
        }
    }
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->gates_applied = n_gates;
    h->gates += double(n_gates);
    return PS_OK;
}

int pauli_sum_truncate(ps_handle* h, double rel_eps, int trunc_mode) {
    if (!h) return fail(PS_ERR_INVALID, "handle is NULL");
    if (h->broken) return fail(PS_ERR_DEVICE, "handle is no longer usable");
    if (trunc_mode == PS_TRUNC_LEARNED && !h->has_scorer)
        return fail(PS_ERR_INVALID, "PS_TRUNC_LEARNED needs pauli_sum_load_scorer first");
    int rc = materialize(h);
    if (rc) return rc;
    if (trunc_mode == PS_TRUNC_NONE || !(rel_eps > 0.0)) return PS_OK;
    if (trunc_mode == PS_TRUNC_LEARNED) {
        const int out = 1 - h->cur, mx_out = 1 - h->mx;
        rc = enqueue_compact(h, h->cur, out, h->mx, mx_out, -1.0, nullptr, 0, false, 0, rel_eps);
        if (rc) return rc;
        h->cur = out;
        h->mx = mx_out;
        return check_no_error(h, "learned truncation");
    }
    h->pend = rel_eps;
    return materialize(h);
}

int expectation_z(ps_handle* h, double* out) {
    if (!h || !out) return fail(PS_ERR_INVALID, "NULL argument");
    if (h->broken) return fail(PS_ERR_DEVICE, "handle is no longer usable");
    int src = h->cur;
    if (h->pend > 0.0) {
        // Pending truncation: only the x == 0 prefix is read.  Its surviving
        // strings are compacted, in order, into the front of the spare state
        // buffer, which then holds exactly the prefix a full truncation pass
        // would have produced; the operator itself stays as stored.
        HIP_TRY(launch_prefix_len(h->ctrl, h->cur, h->buf[h->cur].X, h->stream));
        CompactArgs a{};
        a.ctrl = h->ctrl;
        a.in_buf = h->cur;
        a.out_buf = 1 - h->cur;
        a.mx_in = h->mx;
        a.mx_out = 1 - h->mx;
        a.Xin = h->buf[h->cur].X;
        a.Zin = h->buf[h->cur].Z;
        a.Cin = h->buf[h->cur].C;
        a.Xout = h->buf[1 - h->cur].X;
        a.Zout = h->buf[1 - h->cur].Z;
        a.Cout = h->buf[1 - h->cur].C;
        a.cap = h->cap;
        a.status = h->status;
        a.max_tiles = h->max_tiles;
        a.eps_in = h->pend;
        a.nq = h->nq;
        a.prefix_only = 1;
        LB_RESERVE(h, 1);
        HIP_TRY(launch_compact(a, h->dtype, h->LP, h->stream, h->grid));
        src = 1 - h->cur;
    }
    HIP_TRY(launch_reduce(h->ctrl, src, h->buf[src].X, h->buf[src].C, h->cap, 0, -1.0, h->mx, h->partial,
                          h->red_out, h->dtype, h->LP, h->stream));
    double tmp[kMaxLanes];
    HIP_TRY(hipMemcpyAsync(tmp, h->red_out, h->LP * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    int rc = check_no_error(h, "expectation");
    if (rc) return rc;
    for (int a = 0; a < h->L; ++a) out[a] = tmp[a];
    return PS_OK;
}

int pauli_sum_norm2(ps_handle* h, double* out) {
    if (!h || !out) return fail(PS_ERR_INVALID, "NULL argument");
    if (h->broken) return fail(PS_ERR_DEVICE, "handle is no longer usable");
    // one read of the coefficients; a pending truncation is applied as they are summed
    HIP_TRY(launch_reduce(h->ctrl, h->cur, h->buf[h->cur].X, h->buf[h->cur].C, h->cap, 1, h->pend, h->mx,
                          h->partial, h->red_out, h->dtype, h->LP, h->stream));
    double tmp[kMaxLanes];
    HIP_TRY(hipMemcpyAsync(tmp, h->red_out, h->LP * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    int rc = check_no_error(h, "norm");
    if (rc) return rc;
    for (int a = 0; a < h->L; ++a) out[a] = tmp[a];
    return PS_OK;
}

int pauli_sum_size(ps_handle* h, size_t* n) {
    if (!h || !n) return fail(PS_ERR_INVALID, "NULL argument");
    if (h->broken) return fail(PS_ERR_DEVICE, "handle is no longer usable");
    int rc = materialize(h);
    if (rc) return rc;
    Ctrl c;
    rc = read_ctrl(h, &c);
    if (rc) return rc;
    *n = c.nf[h->cur] + c.nb[h->cur];
    return PS_OK;
}

int pauli_sum_export(ps_handle* h, ps_pauli* keys, void* coeffs, size_t cap, size_t* n) {
    if (!h || !n) return fail(PS_ERR_INVALID, "NULL argument");
    if (h->broken) return fail(PS_ERR_DEVICE, "handle is no longer usable");
    int rc = materialize(h);
    if (rc) return rc;
    Ctrl c;
    rc = read_ctrl(h, &c);
    if (rc) return rc;
    const uint64_t f = c.nf[h->cur], b = c.nb[h->cur];
    *n = f + b;
    if (f + b > cap) return fail(PS_ERR_CAPACITY, "export buffer holds %zu strings, %llu needed", cap,
                                 static_cast<unsigned long long>(f + b));
    if (f + b == 0) return PS_OK;
    if (!keys || !coeffs) return fail(PS_ERR_INVALID, "keys/coeffs NULL");
    std::vector<ulonglong2> X(f + b), Z(f + b);
    const size_t cb = coef_bytes(h);
    std::vector<char> C((f + b) * cb);
    const Buf& B = h->buf[h->cur];
    if (f) {
        HIP_TRY(hipMemcpyAsync(X.data(), B.X, f * 16, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipMemcpyAsync(Z.data(), B.Z, f * 16, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipMemcpyAsync(C.data(), B.C, f * cb, hipMemcpyDeviceToHost, h->stream));
    }
    if (b) {
        HIP_TRY(hipMemcpyAsync(X.data() + f, B.X + (h->cap - b), b * 16, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipMemcpyAsync(Z.data() + f, B.Z + (h->cap - b), b * 16, hipMemcpyDeviceToHost, h->stream));
        HIP_TRY(hipMemcpyAsync(C.data() + f * cb, static_cast<const char*>(B.C) + (h->cap - b) * cb, b * cb,
                               hipMemcpyDeviceToHost, h->stream));
    }
    HIP_TRY(hipStreamSynchronize(h->stream));
    // back run is stored descending
    std::reverse(X.begin() + f, X.end());
    std::reverse(Z.begin() + f, Z.end());
    for (uint64_t i = 0; i < b / 2; ++i)
        std::swap_ranges(C.begin() + (f + i) * cb, C.begin() + (f + i + 1) * cb, C.begin() + (f + b - 1 - i) * cb);
    struct Row {
        U128 x, z;
        uint64_t i;
    };
    std::vector<Row> rows(f + b);
    for (uint64_t i = 0; i < f + b; ++i) {
        rows[i].x = rotl_host({X[i].x, X[i].y}, h->xrot, h->nq);
        rows[i].z = {Z[i].x, Z[i].y};
        rows[i].i = i;
    }
    if (h->xrot != 0) {
        std::sort(rows.begin(), rows.end(), [](const Row& a, const Row& bb) {
            if (a.x.hi != bb.x.hi) return a.x.hi < bb.x.hi;
            if (a.x.lo != bb.x.lo) return a.x.lo < bb.x.lo;
            if (a.z.hi != bb.z.hi) return a.z.hi < bb.z.hi;
            return a.z.lo < bb.z.lo;
        });
    }
    const size_t es = (h->dtype == PS_F64) ? 8 : 4;
    char* dst = static_cast<char*>(coeffs);
    for (uint64_t i = 0; i < f + b; ++i) {
        const Row& r = rows[i];
        keys[i].x[0] = r.x.lo;
        keys[i].x[1] = r.x.hi;
        keys[i].z[0] = r.z.lo;
        keys[i].z[1] = r.z.hi;
        std::memcpy(dst + i * h->L * es, C.data() + r.i * cb, h->L * es);
    }
    return PS_OK;
}

int pauli_sum_set_timing(ps_handle* h, int enable) {
    if (!h) return fail(PS_ERR_INVALID, "handle is NULL");
    HIP_TRY(hipStreamSynchronize(h->stream));
    int rc = ev_collect(h);
    if (rc) return rc;
    h->timing = enable != 0;
    return PS_OK;
}

int pauli_sum_stats(ps_handle* h, ps_stats* out, int reset) {
    if (!h || !out) return fail(PS_ERR_INVALID, "NULL argument");
    Ctrl c;
    int rc = read_ctrl(h, &c);
    if (rc) return rc;
    out->updates = double(c.cnt_updates);
    out->gates = h->gates;
    out->rx_launches = double(c.cnt_rx_launches);
    out->rx_in = double(c.cnt_rx_in);
    out->rx_out = double(c.cnt_rx_out);
    out->rx_ms = h->ms[0];
    out->cliff_launches = double(c.cnt_cliff_launches);
    out->cliff_in = double(c.cnt_cliff_in);
    out->cliff_ms = h->ms[1];
    out->sort_passes = h->sort_passes;
    out->sort_elems = h->sort_elems;
    out->sort_ms = h->ms[2];
    out->bytes_per_string = double(2 * sizeof(ulonglong2) + h->csize);
    out->graph_replays = h->graph_replays;
    out->graph_captures = h->graph_captures;
    out->score_in = double(c.aux[0]);
    out->score_launches = double(c.aux[1]);
    out->score_ms = h->ms[3];
    out->radix_sorts = h->radix_sorts;
    out->run_merges = h->run_merges;
    out->learned_passes = double(c.learned_passes);
    out->learned_fallbacks = double(c.learned_fallbacks);
    out->learned_est = c.learned_est[0];
    out->learned_l1 = c.learned_l1[0];
    out->sort_digit_bits = kSortCandBits[h->sort_last];
    out->sort_items_per_thread = kSortCandIpt[h->sort_last];
    if (reset) {
        h->radix_sorts = h->run_merges = 0;
        h->graph_replays = h->graph_captures = 0;
        h->ms[3] = 0;
        const uint64_t z2[2] = {0, 0};
        HIP_TRY(hipMemcpyAsync(&h->ctrl->aux[0], z2, sizeof z2, hipMemcpyHostToDevice, h->stream));
        const uint64_t z2b[2] = {0, 0};
        HIP_TRY(hipMemcpyAsync(&h->ctrl->learned_passes, z2b, sizeof z2b, hipMemcpyHostToDevice, h->stream));
        c.cnt_updates = c.cnt_rx_in = c.cnt_rx_out = c.cnt_rx_launches = 0;
        c.cnt_cliff_in = c.cnt_cliff_launches = 0;
        HIP_TRY(hipMemcpyAsync(&h->ctrl->cnt_updates, &c.cnt_updates, 6 * sizeof(uint64_t), hipMemcpyHostToDevice,
                               h->stream));
        HIP_TRY(hipStreamSynchronize(h->stream));
        h->ms[0] = h->ms[1] = h->ms[2] = 0;
        h->sort_passes = h->sort_elems = h->gates = 0;
    }
    return PS_OK;
}

int pauli_sum_histogram(ps_handle* h, int lane, const double* edges, int n_bins, int is_signed, uint64_t* counts) {
    int rc = check_histogram_args(h, lane, edges, n_bins, counts);
    if (rc) return rc;
    double* dE = nullptr;
    uint64_t* dC = nullptr;
    if (hipMalloc(reinterpret_cast<void**>(&dE), size_t(n_bins + 1) * 8) != hipSuccess ||
        hipMalloc(reinterpret_cast<void**>(&dC), size_t(n_bins + 2) * 8) != hipSuccess) {
        (void)hipGetLastError();
        if (dE) (void)hipFree(dE);
        return fail(PS_ERR_CAPACITY, "hipMalloc failed for the histogram");
    }
    rc = run_histogram(h, lane, edges, n_bins, is_signed, counts, dE, dC);
    (void)hipFree(dE);
    (void)hipFree(dC);
    return rc;
}

int pauli_sum_histogram_noalloc(ps_handle* h, int lane, const double* edges, int n_bins, int is_signed,
                                uint64_t* counts) {
    int rc = check_histogram_args(h, lane, edges, n_bins, counts);
    if (rc) return rc;
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return fail(PS_ERR_HIP, "hipGetDevice failed");
    if (prev != h->dev) HIP_TRY(hipSetDevice(h->dev));
    void* base = nullptr;
    rc = scratch_address(h->dev, &base);
    if (!rc) {
        double* dE = static_cast<double*>(base);
        uint64_t* dC = static_cast<uint64_t*>(base) + kScratchCountsAt;
        rc = run_histogram(h, lane, edges, n_bins, is_signed, counts, dE, dC);
    }
    if (prev != h->dev) (void)hipSetDevice(prev);
    return rc;
}

int pauli_sum_set_sort_config(ps_handle* h, int digit_bits, int items_per_thread) {
    if (!h) return fail(PS_ERR_INVALID, "NULL argument");
    if (digit_bits == 0 && items_per_thread == 0) {
        h->sort_force = -1;
        return PS_OK;
    }
    for (int c = 0; c < kSortCands; ++c) {
        if (kSortCandBits[c] == digit_bits && kSortCandIpt[c] == items_per_thread) {
            h->sort_force = c;
            return PS_OK;
        }
    }
    return fail(PS_ERR_INVALID, "no radix-sort configuration with %d-bit digits and %d items per thread", digit_bits,
                items_per_thread);
}

int pauli_sum_set_learned(ps_handle* h, double eps_ratio, double tol) {
    if (!h) return fail(PS_ERR_INVALID, "handle is NULL");
    if (!std::isfinite(eps_ratio) || !(eps_ratio > 0.0) || eps_ratio > 1.0)
        return fail(PS_ERR_INVALID, "eps_ratio must be in (0, 1]");
    if (!std::isfinite(tol)) return fail(PS_ERR_NONFINITE, "tol is not finite");
    h->learned_ratio = eps_ratio;
    h->learned_tol = tol;
    return PS_OK;
}

int pauli_sum_set_rx_boundary_prologue(ps_handle* h, int enable) {
    if (!h) return fail(PS_ERR_INVALID, "handle is NULL");
    h->rx_no_prologue = enable == 0;
    drop_graphs(h);  // captured launches carry the setting
    return PS_OK;
}

int pauli_sum_set_lookback_epoch(ps_handle* h, uint32_t epoch) {
    if (!h) return fail(PS_ERR_INVALID, "NULL argument");
    if (h->broken) return fail(PS_ERR_DEVICE, "handle is no longer usable");
    if (epoch < 1 || epoch >= kEpochLimit)
        return fail(PS_ERR_INVALID, "epoch must be in 1..%llu", static_cast<unsigned long long>(kEpochLimit - 1));
    HIP_TRY(hipStreamSynchronize(h->stream));
    HIP_TRY(launch_fill_u64(h->status, 0ull, h->status_words, h->stream));
    HIP_TRY(launch_fill_u64(reinterpret_cast<uint64_t*>(h->desc), 0ull, h->desc_words, h->stream));
    HIP_TRY(hipMemcpyAsync(&h->ctrl->epoch, &epoch, sizeof epoch, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->lb_count = epoch - 1;
    return PS_OK;
}

int pauli_sum_lookback_epoch(ps_handle* h, uint32_t* epoch) {
    if (!h || !epoch) return fail(PS_ERR_INVALID, "NULL argument");
    Ctrl c;
    int rc = read_ctrl(h, &c);
    if (rc) return rc;
    *epoch = c.epoch;
    return PS_OK;
}

int pauli_sum_set_graphs(ps_handle* h, int enable) {
    if (!h) return fail(PS_ERR_INVALID, "NULL argument");
    if (h->broken) return fail(PS_ERR_DEVICE, "handle is no longer usable");
    if (!enable) {
        HIP_TRY(hipStreamSynchronize(h->stream));
        drop_graphs(h);
    }
    h->graphs = enable != 0;
    return PS_OK;
}

int pauli_sum_load_scorer(ps_handle* h, const ps_scorer* sc) {
    if (!h || !sc) return fail(PS_ERR_INVALID, "NULL argument");
    if (!h->has_scorer) {
        int rc = scorer_alloc(&h->scorer);
        if (rc) return rc;
        h->has_scorer = true;
    }
    if (!h->gscore) {
        if (hipMalloc(reinterpret_cast<void**>(&h->gscore), h->cap * sizeof(float)) != hipSuccess) {
            (void)hipGetLastError();
            h->gscore = nullptr;
            return fail(PS_ERR_CAPACITY, "hipMalloc failed for the score array (%zu strings)", h->cap);
        }
    }
    int rc = scorer_copy(&h->scorer, scorer_dev(sc), h->stream);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(h->stream));
    return PS_OK;
}

}  // extern "C"
