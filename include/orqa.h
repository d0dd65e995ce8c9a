/*
 * orqa.h -- C ABI of the MI355X (gfx950) Heisenberg Pauli-propagation library.
 *
 * The library holds an observable O = sum_I O_I sigma_I (Methods, Eq. define_O)
 * as a set of Pauli strings with real coefficients in GPU memory and conjugates
 * it by Pauli rotations exp(-i theta sigma_J / 2) (Appendix A, gate tuple
 * (J, theta_J)) using the coefficient update of Eq. update_rule, with optional
 * dynamic truncation |O_I| <= eps0 * max_I |O_I| after every gate
 * (Eq. truncation1).  <Z> is the sum of the coefficients of strings made of
 * identities and sigma_z only (Eq. magnetization).
 *
 * Pauli strings.  ps_pauli holds the x and z bitmasks of a string on up to 128
 * qubits; qubit q is bit (q & 63) of word (q >> 6).  Letters: I=(0,0), X=(1,0),
 * Y=(1,1), Z=(0,1).  The paper's 2-bit code (h,l) maps to this by x = h xor l,
 * z = h (Methods, Eq. (1)).
 *
 * Coefficient lanes.  Each string carries n_lanes coefficients (1..32).  A lane
 * is an independent operator that shares the key set with the others, with its
 * own initial coefficients and its own angle per gate; the library applies one
 * key pass to all lanes.  Coefficients are passed lane-minor: coeffs[t*n_lanes+a].
 *
 * Precision.  PS_F64 stores and computes coefficients in binary64.  PS_F32
 * stores binary32 coefficients; the per-gate cos/sin products and the sum of the
 * (at most two) contributions to a string are formed in compensated binary32
 * arithmetic (error-free products and two-sum, one final rounding).  Expectation
 * values and norms are always accumulated in binary64.
 *
 * Streams and memory.  All device work of a handle is enqueued on the HIP stream
 * given at creation (NULL: the null stream).  Device memory is owned by the
 * handle and grows on demand.  Calls that return values to the host
 * synchronise that stream.  A handle must not be used by two threads at once.
 *
 * Errors.  Every call returns PS_OK or a negative status; ps_last_error() gives
 * a message for the calling thread's last failure.  Host arrays passed in are
 * only read during the call.
 */
#ifndef ORQA_H
#define ORQA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ps_handle ps_handle;

typedef struct {
    uint64_t x[2];
    uint64_t z[2];
} ps_pauli;

enum {
    PS_OK = 0,
    PS_ERR_INVALID = -1,     /* bad argument: sizes, null pointers, bits above n_qubits */
    PS_ERR_CAPACITY = -2,    /* device memory exhausted or above max capacity */
    PS_ERR_HIP = -3,         /* a HIP runtime call failed */
    PS_ERR_NONFINITE = -4,   /* NaN/Inf coefficient or angle */
    PS_ERR_UNSUPPORTED = -5, /* combination not implemented (see message) */
    PS_ERR_DEVICE = -6       /* a kernel reported an internal failure */
};

enum { PS_F64 = 0, PS_F32 = 1 };
enum { PS_TRUNC_NONE = 0, PS_TRUNC_MAGNITUDE = 1, PS_TRUNC_LEARNED = 2 };

/*
 * pauli_sum_create -- upload an initial operator (Appendix A: the partial
 * representation O = {(I, O_I)} as a list of tuples).
 *   n_qubits  1..128.  Every term must be zero above bit n_qubits-1
 *             (else PS_ERR_INVALID).
 *   n_lanes   1..32 coefficient lanes.
 *   dtype     PS_F64 or PS_F32.
 *   capacity  initial number of strings to reserve (0: library default); the
 *             handle grows beyond it when a gate needs more.
 *   terms     n_terms strings (host).  Duplicates are summed.
 *   coeffs    n_terms*n_lanes binary64 values (host), lane-minor.
 *   hip_stream  hipStream_t to run on, or NULL.
 *   out       receives the handle.
 */
int pauli_sum_create(int n_qubits, int n_lanes, int dtype, size_t capacity,
                     const ps_pauli* terms, const double* coeffs, size_t n_terms,
                     void* hip_stream, ps_handle** out);

/* pauli_sum_destroy -- free all device memory of the handle (NULL is a no-op). */
int pauli_sum_destroy(ps_handle* h);

/*
 * apply_rotation_layer -- conjugate the operator by n_gates Pauli rotations in
 * the order given (Heisenberg order: gate 0 acts on the observable first), each
 * O <- U^dag O U with U = exp(-i theta sigma_J / 2), coefficient update of
 * Eq. update_rule (Algorithm 1, gate loop).
 *   gens     n_gates generators sigma_J (host).
 *   thetas   n_gates*n_lanes angles (host), lane-minor.  Angles within
 *            1e-12*max(1,|theta|) of a multiple of pi/2 use exact cos/sin in
 *            {0,+-1}; a zero factor creates no string.
 *   rel_eps  eps0 of Eq. truncation1: after every gate drop every string whose
 *            coefficient satisfies |O_I,a| <= rel_eps * max_I |O_I,a| in every
 *            lane a (max over the whole operator after that gate).  rel_eps <= 0
 *            keeps every generated string, exact zeros included.
 *   trunc_mode  PS_TRUNC_MAGNITUDE (rule above), PS_TRUNC_NONE (rel_eps
 *            ignored), PS_TRUNC_LEARNED (rule above after every gate, plus
 *            the learned rule, see ps_scorer_create, once per run of Clifford
 *            gates, i.e. once per Trotter step; needs a loaded scorer).
 * Fast paths: runs of Clifford gates whose generators hold only Z letters
 * (e.g. RZZ(-pi/2) layers) are fused into one pass plus one re-sort; sigma_x
 * rotations on consecutive qubits q, q+1, ... (each layer ascending, starting at
 * qubit 0) run as one streaming pass per gate.  Any other generator takes the
 * general path: a branch pass (parent part and child per string), a sort by
 * key (inside each x-group for Z-only generators; a gather and pairwise merge
 * of the branch's sorted runs when the generator flips few key bits; else the
 * radix sort) and a pass summing the entries of equal keys.
 * On PS_ERR_CAPACITY the gates before the failing one have been applied
 * (pauli_sum_gates_applied tells how many) and the handle stays usable.
 */
int apply_rotation_layer(ps_handle* h, const ps_pauli* gens, const double* thetas,
                         size_t n_gates, double rel_eps, int trunc_mode);

/* Number of gates of the last apply_rotation_layer call that were applied. */
int pauli_sum_gates_applied(ps_handle* h, size_t* n);

/*
 * pauli_sum_truncate -- one truncation of the current operator with the rule
 * of Eq. truncation1 (Algorithm 1, truncation loop).  Named with the library
 * prefix so it does not clash with POSIX truncate(2).
 */
int pauli_sum_truncate(ps_handle* h, double rel_eps, int trunc_mode);

/* expectation_z -- <0|O|0> per lane (Eq. magnetization), binary64 (host out[n_lanes]). */
int expectation_z(ps_handle* h, double* out);

/* pauli_sum_size -- number of strings held (|O|, the effective complexity, Methods). */
int pauli_sum_size(ps_handle* h, size_t* n);

/*
 * pauli_sum_norm2 -- sum_I O_I,a^2 per lane, binary64 (host out[n_lanes]).
 * With the coefficients of Eq. define_O being the normalised traces on the
 * left of Eq. update_rule, this is Tr[O^2] / 2^n.  Every gate maps each pair
 * {I, I xor J} by a rotation (Eq. update_rule), so the value is conserved
 * without truncation; truncation (Eq. truncation1) lowers it by the squares
 * it drops (the value is that of the operator after the last gate's
 * truncation).
 */
int pauli_sum_norm2(ps_handle* h, double* out);

/*
 * pauli_sum_export -- the operator as the list of tuples (I, O_I) of its
 * strings (Appendix A, the representation each process holds), copied to the
 * host: up to cap strings, sorted by (x[1], x[0], z[1], z[0]) ascending.
 * coeffs receives cap*n_lanes values of the handle's dtype (double for
 * PS_F64, float for PS_F32), lane-minor.  *n receives the number of strings
 * held; if it exceeds cap nothing is written and PS_ERR_CAPACITY is returned.
 * pauli_sum_create of the exported tuples (same dtype) restores the same
 * strings and coefficients (checkpoint and resume).
 */
int pauli_sum_export(ps_handle* h, ps_pauli* keys, void* coeffs, size_t cap, size_t* n);

/*
 * Learned truncation scorer (PS_TRUNC_LEARNED).  A small network (160 -> 128
 * -> 128 -> 1, GELU, bf16 weights, fp32 accumulation) maps a string's key to
 * y = log10 of the predicted weight g_I with which the string still reaches
 * <Z> after the rest of the circuit; learned truncation drops strings with
 * |O_I,a| * min(1, 10^y) <= rel_eps * max_I |O_I,a| in every lane.  The paper
 * uses the magnitude rule (Eq. truncation1) and names tailored truncation as
 * future work (Conclusion; Appendix D); this is that extension, with the
 * magnitude rule kept as its fallback.
 *
 * Features: feature f counts the qubits of qmask[f] (two words) that carry
 * letter letters[f] (0 X, 1 Y, 2 Z, 3 any non-identity), times scales[f].
 * Parameters: one fp32 vector of 37249 values, W1 (128x160 row major), b1
 * (128), W2 (128x128), b2 (128), W3 (128), b3 (1).
 *
 * ps_scorer_create      allocate a scorer for n_qubits with the 160 feature
 *                       definitions (host arrays: qmask 320 words, letters
 *                       160, scales 160); parameters start at zero.
 * ps_scorer_set_params  upload parameters (resets the Adam moments).
 * ps_scorer_get_params  download parameters.
 * ps_scorer_set_data    upload a training set: n keys and n fp32 targets.
 * ps_scorer_forward     network outputs y (host out[n], may be NULL) and the
 *                       bf16 features (host out[n*160], may be NULL) of the
 *                       training set.
 * ps_scorer_loss_grad   mean squared error of y against the targets and its
 *                       gradient (host out[37249], may be NULL).
 * ps_scorer_adam_step   one Adam step (beta 0.9/0.999, eps 1e-8) with the
 *                       last gradient.
 * pauli_sum_load_scorer copy the scorer's network into the handle (the scorer
 *                       may be destroyed afterwards).
 */
/*
 * pauli_sum_histogram -- the Pauli-string density of Appendix D: counts of the
 * coefficients of lane `lane` rescaled by their largest magnitude,
 * x = O_I / max_I |O_I| (is_signed != 0) or |O_I| / max_I |O_I| (is_signed == 0),
 * over the bins [edges[k], edges[k+1]) for k < n_bins - 1 and the closed last
 * bin [edges[n_bins-1], edges[n_bins]].  edges (host, n_bins + 1 values,
 * strictly increasing, 1 <= n_bins <= 4096); bin membership is decided by
 * comparing the coefficient with max|O| * edges[k] in binary64.  counts (host
 * out, n_bins + 2): the bins, then the values below edges[0], then those above
 * edges[n_bins].  Strings a pending truncation drops are not counted (the
 * counts equal those of the truncated operator).  Device memory for the
 * edges and counters is allocated and freed by each call.
 * Errors: PS_ERR_INVALID (NULL pointer, lane out of range, n_bins outside
 * 1..4096, edges not increasing), PS_ERR_NONFINITE (an edge), PS_ERR_CAPACITY
 * (hipMalloc failed); the operator is never changed.
 */
int pauli_sum_histogram(ps_handle* h, int lane, const double* edges, int n_bins, int is_signed, uint64_t* counts);

/*
 * pauli_sum_histogram_noalloc -- pauli_sum_histogram for callers that cannot
 * allocate device memory (code that may run under HIP graph capture set-up,
 * tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * counts and errors, but the call allocates and frees nothing: its edges and
 * counters (at most 4096 bins, 64 KiB and a bit) live in one fixed device
 * array of the library, one copy per GPU, held until the process ends.  The
 * counters are cleared by every call.  All calls on one GPU share that array:
 * calls that overlap in time on the same GPU (two host threads, or handles on
 * two streams) race and may return wrong counts.  n_bins above 4096:
 * PS_ERR_INVALID.
 */
int pauli_sum_histogram_noalloc(ps_handle* h, int lane, const double* edges, int n_bins, int is_signed,
                                uint64_t* counts);

/*
 * pauli_sum_set_sort_config -- digit width and tile size of the radix sort
 * (the re-sort after a Clifford layer, Eq. (u), when its x-groups are too large
 * for the in-group sort, and the sort of general gates, Eq. update_rule, whose
 * generators flip too many key bits for the run merge).
 * (digit_bits, items_per_thread) is one of (8, 8), (8, 16), (7, 16), (6, 16),
 * (7, 8), (6, 8); a tile holds 256 * items_per_thread strings.  (0, 0), the
 * default, tunes online: the first sorts of each size class (powers of two of
 * the string count, from 2^16) and key kind time each configuration once, and
 * later sorts of that class use the fastest.  Every configuration sorts the
 * same keys into the same order, so results do not depend on this setting.
 * Errors: PS_ERR_INVALID for any other pair.
 */
int pauli_sum_set_sort_config(ps_handle* h, int digit_bits, int items_per_thread);

/*
 * pauli_sum_set_graphs -- with enable != 0, every run of consecutive RX gates
 * in a layer (e.g. the RX half of a Trotter step) is captured once into a HIP
 * graph and replayed when the same gates meet the same buffers again, so a
 * layer of 127 rotations costs one graph launch instead of 254 kernel
 * launches.  Results are identical to the eager path.  Graphs are not used
 * while timing is on, and are dropped when the capacity grows (the buffers
 * move).  Capture uses a stream of the handle's own; replays go to the
 * handle's stream.  enable == 0 drops the cached graphs.
 */
int pauli_sum_set_graphs(ps_handle* h, int enable);

/*
 * Look-back epoch (for tests of its guard).  The single-pass kernels that
 * assign output offsets (stream compaction, Algorithm 1's truncation loop,
 * and the merge of Eq. update_rule) publish per-tile status words tagged with
 * the low 24 bits of a launch counter, the epoch; words of other launches
 * read as not ready, so the words are never cleared between launches.  The
 * library clears them and restarts the epoch at 1 before the tag can wrap.
 *   pauli_sum_set_lookback_epoch  clear the status words and restart the
 *                                 epoch at `epoch` (1 .. 2^24 - 3, else
 *                                 PS_ERR_INVALID), e.g. just below the wrap.
 *   pauli_sum_lookback_epoch      read the current epoch (host out).
 */
int pauli_sum_set_lookback_epoch(ps_handle* h, uint32_t epoch);
int pauli_sum_lookback_epoch(ps_handle* h, uint32_t* epoch);

/*
 * RX tile boundaries (for tests of both paths).  The streaming pass of a
 * sigma_x rotation (Eq. update_rule) cuts its merged order into tiles; the
 * grid first finds every tile boundary (each stored as words tagged with the
 * launch's epoch), and a tile whose boundaries have not arrived in time
 * finds them itself.  enable == 0 skips the first step, so that every tile
 * finds its own boundaries; results are identical either way.
 */
int pauli_sum_set_rx_boundary_prologue(ps_handle* h, int enable);

/*
 * pauli_sum_set_learned -- the learned rule's threshold and its fallback to
 * magnitude truncation (Eq. truncation1).  The learned rule of
 * PS_TRUNC_LEARNED drops a string the magnitude rule keeps when
 * |O_I,a| * min(1, 10^y) <= eps_ratio * rel_eps * max_I |O_I,a| in every lane
 * (eps_ratio in (0, 1], default 1).  Before each learned pass the library
 * estimates the error of those extra drops per lane,
 * sqrt(sum over them of (|O_I,a| min(1, 10^y))^2) (their contributions to
 * <Z> with independent signs); with tol > 0, a pass whose estimate exceeds
 * tol in some lane applies the magnitude rule alone instead.  tol <= 0 (the
 * default): never fall back.  ps_stats reports the learned passes, how many
 * fell back, and the last estimate with its sum of |O_I,a| min(1, 10^y)
 * (lane 0).  Errors: PS_ERR_INVALID (eps_ratio outside (0, 1]),
 * PS_ERR_NONFINITE (tol).
 */
int pauli_sum_set_learned(ps_handle* h, double eps_ratio, double tol);

typedef struct ps_scorer ps_scorer;
int ps_scorer_create(int n_qubits, const uint64_t* qmask, const uint8_t* letters, const float* scales,
                     void* hip_stream, ps_scorer** out);
int ps_scorer_destroy(ps_scorer* s);
int ps_scorer_set_params(ps_scorer* s, const float* params, size_t n);
int ps_scorer_get_params(ps_scorer* s, float* params, size_t n);
int ps_scorer_set_data(ps_scorer* s, const ps_pauli* keys, const float* targets, size_t n);
int ps_scorer_forward(ps_scorer* s, float* y, uint16_t* features);
int ps_scorer_loss_grad(ps_scorer* s, double* loss, float* grad);
int ps_scorer_adam_step(ps_scorer* s, float lr);
int pauli_sum_load_scorer(ps_handle* h, const ps_scorer* s);

/*
 * Counters and timing for measurement.  Counters accumulate since creation or
 * the last reset; kernel times are only collected while timing is enabled
 * (HIP events around each launch on the handle's stream, read back at the
 * synchronisation points of apply_rotation_layer).
 *   updates        sum over gates of the number of strings the gate read
 *                  (|O| before the gate, the paper's per-gate cost measure)
 *   gates          gates applied
 *   rx_launches    streaming RX merge launches; rx_in / rx_out strings read /
 *                  written by them; rx_ms their summed kernel time
 *   cliff_launches fused Clifford / compaction launches; cliff_ms their time
 *                  plus that of the branch and equal-key passes of general
 *                  gates
 *   sort_passes    sort passes (in-group sorts, radix passes, run gathers and
 *                  merge levels), sort_elems the strings they moved, sort_ms
 *                  their time
 *   bytes_per_string  key + coefficient bytes of one stored string
 *   graph_replays, graph_captures  runs of RX gates replayed from / captured
 *                  into HIP graphs (pauli_sum_set_graphs)
 *   score_launches, score_in, score_ms  learned-scorer launches, strings
 *                  scored and their kernel time (PS_TRUNC_LEARNED)
 *   radix_sorts    radix sorts run (re-sorts whose x-groups did not fit the
 *                  in-group sort, and sorts of general gates);
 *                  sort_digit_bits, sort_items_per_thread the configuration
 *                  of the last one (pauli_sum_set_sort_config)
 *   run_merges     general gates sorted by gathering their runs (parents;
 *                  children by class) and merging them pairwise
 *   learned_passes, learned_fallbacks, learned_est, learned_l1  learned
 *                  truncation passes, those that fell back to the magnitude
 *                  rule, and the last pass's error estimate (lane 0; see
 *                  pauli_sum_set_learned)
 */
typedef struct {
    double updates, gates;
    double rx_launches, rx_in, rx_out, rx_ms;
    double cliff_launches, cliff_in, cliff_ms;
    double sort_passes, sort_elems, sort_ms;
    double bytes_per_string;
    double graph_replays, graph_captures;
    double score_launches, score_in, score_ms;
    double radix_sorts, sort_digit_bits, sort_items_per_thread;
    double run_merges;
    double learned_passes, learned_fallbacks, learned_est, learned_l1;
} ps_stats;

int pauli_sum_set_timing(ps_handle* h, int enable);
int pauli_sum_stats(ps_handle* h, ps_stats* out, int reset);

/* Message for the calling thread's last non-OK status (never NULL). */
const char* ps_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ORQA_H */
