// Internal types shared by the gfx950 kernels and the host engine.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace orqa {

constexpr int kMaxLanes = 32;
constexpr int kMaxCliffGens = 512;  // Clifford generators fused into one pass
constexpr int kMaxCliffGroups = 32; // offset groups of weight-2 generators (CliffGroup)

// Error bits raised by kernels in Ctrl::err.
constexpr uint32_t kErrCapacity = 1u;
constexpr uint32_t kErrLookback = 2u;
constexpr uint32_t kErrInternal = 4u;  // inconsistent tile split (never expected)

// Tile sizes.  An RX tile covers kRxTile merged positions; pair-preserving
// boundary adjustment can move either end by one, so a tile holds at most
// kRxTile + 1 <= kRxTileMax strings.
constexpr int kThreads = 256;
constexpr int kRxIPT = 3;
constexpr int kRxTileMax = kThreads * kRxIPT;  // 768
constexpr int kRxTile = kRxTileMax - 2;        // 766
constexpr int kRxHold = 4;  // output entries per thread an RX workgroup holds in registers across tiles
constexpr int kCompactIPT = 4;
constexpr int kCompactTile = kThreads * kCompactIPT;  // 1024
constexpr int kSortIPT = 8;                     // smallest items per thread of a sort pass
constexpr int kSortTile = kThreads * kSortIPT;  // 2048: smallest sort tile (sizes the status words)
constexpr int kSortMaxPasses = 48;              // 2 x ceil(128 / 6) digits at the narrowest width
constexpr int kReduceBlocks = 512;

// Device-resident control block of a handle.  The two state buffers each hold
// a "virtual array": a front run at [0, nf) ascending and a back run stored
// descending from the end of the buffer, [cap-nb, cap).  Logical element i is
// physical i for i < nf and cap-1-(i-nf) otherwise.
constexpr uint32_t kTileStreams = 8;

struct Ctrl {
    uint64_t nf[2];
    uint64_t nb[2];
    uint64_t maxbits[2][kMaxLanes];  // max |c| per lane as binary64 bits, two slots
    uint32_t tile_counter;           // dynamic tile index of the running look-back kernel
    uint32_t done_counter;           // workgroups finished (last one resets the two counters)
    uint32_t epoch;                  // look-back status generation, bumped per look-back launch
    uint32_t err;                    // kErr* bits
    uint64_t need;                   // strings a failed stage needed
    uint64_t stages_done;            // stages finished without error since the host reset it
    uint64_t prefix_len;             // length of the x == 0 prefix (expectation)
    uint64_t nranks;                 // x-groups counted by the last Clifford pass
    uint64_t cnt_updates;            // sum over gates of strings read
    uint64_t cnt_rx_in, cnt_rx_out, cnt_rx_launches;
    uint64_t cnt_cliff_in, cnt_cliff_launches;
    uint64_t aux[4];
    // learned truncation: per lane, the estimated error of the strings that
    // only the learned rule drops, sqrt(sum (|c| min(1, 10^y))^2), and its
    // sum of |c| min(1, 10^y); passes that fell back to the magnitude rule
    double learned_est[kMaxLanes];
    double learned_l1[kMaxLanes];
    uint64_t learned_passes, learned_fallbacks;
    // tile counters of the look-back kernels, one per workgroup stream
    // (blockIdx modulo kTileStreams), each on a cache line of its own
    alignas(128) uint32_t tile_ctr[kTileStreams][32];
};

// Tile boundary of an RX merge: the split of merged position b.
struct TileDesc {
    uint64_t posA, posB, hm, he;
};

// Per-gate trigonometry (per lane), exact at Clifford angles.  The fp32 form
// splits each value into hi + lo.
struct GateTrig {
    double cs[kMaxLanes], sn[kMaxLanes];
    float cs_hi[kMaxLanes], cs_lo[kMaxLanes], sn_hi[kMaxLanes], sn_lo[kMaxLanes];
    int any_c, any_s;
    int zword, zbit;  // location of z_j of the rotated qubit j
};

// A Z-only Clifford generator: z mask and the action on anticommuting strings.
// kodd: theta = +-pi/2 (mod 2pi): key becomes K = I xor J with factor
// sign(B(K,J)) * sin(theta); otherwise theta = pi (mod 2pi): factor -1.
struct CliffGen {
    uint64_t z0, z1;
    uint32_t kodd;
    uint32_t neg;  // kodd: sin(theta) = -1; else: cos(theta) = -1
};

// Weight-2 Z-only generators Z_a Z_(a+d) of one Clifford run that share the
// qubit offset d, as masks over the lower qubit a: k for those with
// sin(theta) = +-1 (the string is multiplied by Z_a Z_(a+d)), n for those
// whose factor is negative.  A run's generators all commute, so the pass
// applies them in any grouping.
struct CliffGroup {
    uint64_t k0, k1;
    uint64_t n0, n1;
    uint32_t d;
    uint32_t pad;
};

struct Buf {
    ulonglong2* X;  // stored (rotated) x mask
    ulonglong2* Z;
    void* C;        // cap x lanes_pad coefficients
};

struct RxArgs {
    Ctrl* ctrl;
    int in_buf, out_buf, mx_in, mx_out;
    const ulonglong2* Xin;
    const ulonglong2* Zin;
    const void* Cin;
    ulonglong2* Xout;
    ulonglong2* Zout;
    void* Cout;
    uint64_t cap;
    TileDesc* desc;    // tile boundaries of the input (found by the kernel itself), ntiles + 1
    uint64_t* status;  // 2 x (max_tiles + max_tiles / 64 + 2): tile words, then group words, per channel
    uint64_t max_tiles;
    double eps_in;     // pending truncation of the input (<= 0: none)
    int nq;
    int no_prologue;   // tiles find their own boundaries (tests of that path)
};

struct CompactArgs {
    Ctrl* ctrl;
    int in_buf, out_buf, mx_in, mx_out;
    const ulonglong2* Xin;
    const ulonglong2* Zin;
    const void* Cin;
    ulonglong2* Xout;
    ulonglong2* Zout;
    void* Cout;
    uint32_t* rank_out;  // may be null
    uint64_t cap;
    uint64_t* status;    // 2 x max_tiles
    uint64_t max_tiles;
    double eps_in;
    int nq, xrot;
    const CliffGen* gens;   // generators applied one by one
    int ngens;
    const CliffGroup* groups;  // weight-2 generators by qubit offset
    int ngroups;
    int groups_neg_is_k;       // every group's n masks equal its k masks
    int gate_count;      // gates this pass stands for (measurement counters)
    const float* gscore;  // learned truncation: log10 predicted weight per input string, or null
    double eps_learned;
    double learned_tol;   // fall back to the magnitude rule when some lane's learned_est exceeds it (<= 0: never)
    // prefix_only: compact only the first ctrl->prefix_len strings of the
    // input (the x == 0 prefix) for a readout, with no other effect on the
    // handle: no maxima, counters or sizes of the operator are touched; the
    // result's length replaces ctrl->prefix_len and becomes the size of the
    // output buffer
    int prefix_only;
};

// A radix-sort key is read as one integer whose 64-bit words, least
// significant first, are z.x, z.y, the x-group rank, x.x, x.y; a digit is the
// `w` bits (1..8) starting at bit `lo` of that integer.
struct SortPlan {
    int npass;
    uint16_t lo[kSortMaxPasses];
    uint8_t w[kSortMaxPasses];
};

struct SortPassArgs {
    Ctrl* ctrl;
    uint64_t n;
    int lo, w;                   // digit bits [lo, lo + w) of the key
    const uint32_t* digit_base;  // 2^w exclusive bucket starts for this digit
    const uint32_t* Rs;          // NULL: no rank in the key (not moved either)
    const ulonglong2* Zs;
    const ulonglong2* Xs;
    const void* Cs;
    uint32_t* Rd;
    ulonglong2* Zd;
    ulonglong2* Xd;
    void* Cd;
    uint64_t* status;        // max_tiles x 256
    uint64_t max_tiles;
    int dst_buf;
    // binary32 general gates: the low words of the branch's products (n x
    // lanes), moved with the strings; NULL otherwise
    const float* Ls;
    float* Ld;
};

// Host-side launchers (orqa_kernels.hip), dispatching on dtype and padded lanes.
hipError_t launch_rx(const RxArgs& a, const GateTrig& g, int dtype, int lp, hipStream_t s, int grid);
int rx_blocks_per_cu(int dtype, int lp);
hipError_t launch_compact(const CompactArgs& a, int dtype, int lp, hipStream_t s, int grid);
hipError_t launch_sort_hist(Ctrl* ctrl, int buf, const uint32_t* R, const ulonglong2* Z, const ulonglong2* X,
                            const SortPlan& plan, uint32_t* hist, hipStream_t s, int grid);
hipError_t launch_sort_pass(const SortPassArgs& a, int ipt, int dtype, int lp, hipStream_t s, int grid);

// Re-sort after a Clifford layer when every x-group is small: each group is
// sorted by z inside one workgroup, in place of the groups' positions.
constexpr int kGsThreads = 512;
constexpr int kGsTile = 1024;                  // positions whose groups a workgroup sorts
constexpr int kGsMaxGroup = 3072;              // larger groups: radix-sort fallback
constexpr int kGsCap = kGsTile + kGsMaxGroup;  // strings staged per tile
constexpr int kGsIPT = kGsCap / kGsThreads;
struct GroupSortArgs {
    Ctrl* ctrl;
    int in_buf, out_buf;
    const ulonglong2* Xs;
    const ulonglong2* Zs;
    const void* Cs;
    ulonglong2* Xd;
    ulonglong2* Zd;
    void* Cd;
    const float* Ls;  // low words moved with the strings (binary32 general gates), or NULL
    float* Ld;
    int xor_order;    // every group is a z-sorted run XORed with one mask (after a Clifford run)
};
hipError_t launch_group_sort(const GroupSortArgs& a, int dtype, int lp, hipStream_t s, int grid);

// General Pauli rotation (any sigma_J): branch every string into its parent
// part and, when it anticommutes with sigma_J, its child I xor J (unsorted,
// true x); after a full (x, z) sort, merge the at most two entries per key.
constexpr int kGenIPT = 4;
constexpr int kGenTile = kThreads * kGenIPT;
struct GenArgs {
    Ctrl* ctrl;
    int in_buf, out_buf, mx_in, mx_out;
    const ulonglong2* Xin;
    const ulonglong2* Zin;
    const void* Cin;
    ulonglong2* Xout;
    ulonglong2* Zout;
    void* Cout;
    uint64_t cap;
    uint64_t* status;
    uint64_t max_tiles;
    double eps_in;  // pending truncation threshold of the input (<= 0: none)
    int xrot, nq;
    uint64_t xj0, xj1, zj0, zj1;  // the generator sigma_J
    // run tags (NULL: none): 0 for a parent, 1 + class for a child, the class
    // being the parent's bits at the generator's run_bits key positions
    // (run_pos, in z when run_isz, else in the stored x)
    uint32_t* Tout;
    int run_bits;
    uint8_t run_pos[6];
    uint8_t run_isz[6];
    // binary32: the branch writes each output as an unevaluated pair, the
    // rounded product in Cout and its low word in Lout (the exact product of
    // the split cos / sin, Arith<float>); the equal-key pass sums the pairs of
    // a key with two-sum and rounds once (Lin).  NULL for binary64.
    float* Lout;
    const float* Lin;
};
constexpr int kRunMaxBits = 6;  // at most 1 + 2^6 sorted runs per general gate

// Merge of pairs of adjacent sorted runs (general gates): pair p merges
// [a0, a0 + na) and [a0 + na, a0 + na + nb) of the source into [a0, ...) of
// the destination; its output tiles are tile0 .. tile0 + ceil((na+nb)/T) - 1.
constexpr int kMergeIPT = 4;
constexpr int kMergeTile = kThreads * kMergeIPT;  // 1024
constexpr int kMergeMaxPairs = 64;
struct MergePair {
    uint64_t a0, na, nb, tile0;
};
struct MergeArgs {
    Ctrl* ctrl;
    int npairs, dst_buf;
    uint64_t ntiles, n;
    MergePair pairs[kMergeMaxPairs];
    const ulonglong2* Xs;
    const ulonglong2* Zs;
    const void* Cs;
    ulonglong2* Xd;
    ulonglong2* Zd;
    void* Cd;
    uint64_t* split;  // per tile: A elements before its first output (within its pair)
    const float* Ls;  // low words moved with the strings (binary32 general gates), or NULL
    float* Ld;
};
hipError_t launch_merge_pairs(const MergeArgs& a, int dtype, int lp, hipStream_t s);
hipError_t launch_gen_branch(const GenArgs& a, const GateTrig& g, int dtype, int lp, hipStream_t s, int grid);
hipError_t launch_gen_reduce(const GenArgs& a, int dtype, int lp, hipStream_t s, int grid);

// Coefficient histogram (Pauli-string density, Appendix D).  Thresholds are
// formed on the device as M * edge_k (binary64 products, M = the lane's max
// |c| in ctrl->maxbits[mx]); strings a pending truncation would drop
// (|c| <= eps_pend * max |c| in every lane) are not counted.
constexpr int kHistMaxBins = 4096;
struct HistArgs {
    const Ctrl* ctrl;
    int buf, mx;
    const void* C;
    uint64_t cap;
    int lane, nbins, is_signed;
    double eps_pend;       // pending truncation of the operator (<= 0: none)
    const double* edges;   // nbins + 1, increasing (device)
    uint64_t* counts;      // nbins + 2 (device, zeroed by the caller)
};
hipError_t launch_histogram(const HistArgs& a, int dtype, int lp, hipStream_t s, int grid);

#define ORQA_DISPATCH(DTYPE, LP, F)                      \
    do {                                                 \
        if ((DTYPE) == 0) {                              \
            switch (LP) {                                \
                case 1: F(double, 1); break;             \
                case 2: F(double, 2); break;             \
                case 4: F(double, 4); break;             \
                case 8: F(double, 8); break;             \
                case 16: F(double, 16); break;           \
                case 32: F(double, 32); break;           \
                default: return hipErrorInvalidValue;    \
            }                                            \
        } else {                                         \
            switch (LP) {                                \
                case 1: F(float, 1); break;              \
                case 2: F(float, 2); break;              \
                case 4: F(float, 4); break;              \
                case 8: F(float, 8); break;              \
                case 16: F(float, 16); break;            \
                case 32: F(float, 32); break;            \
                default: return hipErrorInvalidValue;    \
            }                                            \
        }                                                \
    } while (0)

// mode 0: <Z> over the x == 0 prefix of buffer buf (no pending truncation:
// compact the prefix first); mode 1: sum of c^2 over the buffer, skipping the
// strings a pending truncation eps_pend (max slot mx) drops.
hipError_t launch_reduce(Ctrl* ctrl, int buf, const ulonglong2* X, const void* C, uint64_t cap, int mode,
                         double eps_pend, int mx, double* partial, double* out, int dtype, int lp, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s);
// Estimated error of the learned rule on buffer buf (into ctrl->learned_est
// and learned_l1): strings the magnitude rule keeps (|c| > eps_pend * M in
// some lane) but the learned rule drops (|c| min(1, 10^y) <= eps_learned * M
// in every lane).  partial: kReduceBlocks x 2 x lanes doubles.
hipError_t launch_learned_estimate(Ctrl* ctrl, int buf, const void* C, const float* gscore, uint64_t cap,
                                   double eps_pend, double eps_learned, int mx, double* partial, int dtype, int lp,
                                   hipStream_t s);
// Length of the x == 0 prefix of buffer buf into ctrl->prefix_len.
hipError_t launch_prefix_len(Ctrl* ctrl, int buf, const ulonglong2* X, hipStream_t s);

}  // namespace orqa
