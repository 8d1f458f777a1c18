/*
 * tn.h -- C ABI of the sliced big-head tensor-network contraction on MI355X.
 *
 * The library computes, for a random quantum circuit U on n qubits, the
 * amplitudes of all 2^n2 bitstrings that agree with fixed bits s1 on the n1
 * closed qubits and take every value on the n2 open qubits:
 *
 *     A[s2] = <s1; s2| U |0^n>,
 *
 * by contracting the circuit's tensor network (single-qubit gates absorbed
 * into two-qubit gates; section "Computing bitstring probabilities"), sliced
 * into 2^k independent subtasks whose results are summed (appendix A,
 * "Dynamic slicing"), with the big-head split of the network into a head of
 * closed qubits and a tail of open qubits joined by a small cut (section
 * "Big-head simulation of quantum circuits").  XEB (Eq. 1) and the marginal
 * and conditional probabilities (appendix C) are computed from the result.
 *
 * Conventions shared by every call:
 *  - Every function returns tn_status: 0 on success, a negative code on
 *    failure; tn_last_error() then returns a thread-local message.  No call
 *    aborts the process or lets a C++ exception escape.
 *  - Complex numbers are interleaved (re, im).  Device buffers named d_* are
 *    device pointers allocated by the caller (e.g. through PyTorch) on the
 *    current HIP device; h_* are host pointers owned by the caller.
 *  - Calls taking a hip_stream (a hipStream_t, NULL = the null stream) are
 *    asynchronous on that stream unless stated otherwise.
 *  - Qubit q is bit (n-1-q) of a full basis index; the amplitude index of
 *    s2 takes the open qubits in ascending id, the first open qubit as the
 *    most significant bit.
 *  - Edge (q, t) is the wire of qubit q after its t-th two-qubit gate
 *    (t = 0, 1, ...); (q, -1) is the wire of a qubit with no two-qubit gate.
 *    Single-qubit gates are absorbed forward into the next two-qubit gate on
 *    their qubit, trailing ones backward into the last, |0> into the first
 *    and the projector <s1_q| into the last two-qubit gate of qubit q.
 *  - Slice j fixes the i-th sliced edge to bit i of j.
 *  - A plan keeps device state (leaves, slice-invariant tensors, the tail of
 *    the big-head split, profiling events): calls on one plan must not run
 *    concurrently, from several host threads or on several streams at once.
 *    Different plans are independent; planning itself is re-entrant.
 */
#ifndef TN_H
#define TN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tn_plan_s* tn_plan_t;

typedef enum {
    TN_OK = 0,
    TN_EINVAL = -1,        /* bad argument (see each call) */
    TN_ENOMEM = -2,        /* host or device allocation failed */
    TN_EDEVICE = -3,       /* a HIP call failed */
    TN_ESTATE = -4,        /* call made in a state that does not allow it */
    TN_EUNSUPPORTED = -5   /* option with no implementation */
} tn_status;

typedef enum {
    TN_C64 = 0,        /* complex64 storage, FP32 MFMA (the paper's precision) */
    TN_C128 = 1,       /* complex128 storage and arithmetic (FP64 recontraction) */
    TN_SPLIT_FP16 = 2, /* complex64 storage; dense steps as hi/lo FP16 pairs on FP16 MFMA
                          (3 products), FP32 accumulation, per-tensor power-of-two scaling */
    TN_BF16 = 3        /* complex64 storage; dense steps on BF16 MFMA (1 product),
                          FP32 accumulation, per-tensor power-of-two scaling */
} tn_precision;

/* One gate: q1 = -1 for a single-qubit gate.  Matrix row-major, row = output
 * basis state, column = input; two-qubit basis |q0 q1> with q0 the more
 * significant bit.  2x2 gates use the first 4 entries. */
typedef struct {
    int32_t q0, q1;
    double re[16], im[16];
} tn_gate;

/* A circuit: gates in time order, initial state |0^n>. */
typedef struct {
    int32_t n_qubits;
    int32_t n_gates;
    const tn_gate* gates;
} tn_circuit;

typedef struct {
    int32_t qubit, segment;   /* edge (q, t) */
} tn_edge;

/* A contraction tree as SSA pairs: leaves are 0..L-1 in network order (one
 * per two-qubit gate in time order, then one per gate-less qubit in id
 * order); step s creates node L+s from nodes lhs[s] and rhs[s]. */
typedef struct {
    int32_t n_steps;
    const int32_t* lhs;
    const int32_t* rhs;
} tn_tree;

typedef struct {
    tn_precision prec;
    int32_t max_log2_size;   /* memory target: largest intermediate of one slice
                                (log2 elements); slicing continues until met */
    int32_t n_slice_edges;   /* >= 0: slice at least this many edges; -1: target only */
    int32_t batch_log2;      /* slices contracted together per launch sequence
                                (log2); -1 = chosen by the planner */
    int32_t branch_merge;    /* 1 = merge small branches before large steps */
    int32_t bighead;         /* 1 = big-head split (section "Big-head simulation"): a tail
                                holding every open leg is cut off with n_c <= 28 cut legs;
                                all sliced edges lie in the head, whose result v_head[c] is
                                what the slices sum into (the accumulator has 2^n_c
                                entries).  tn_amplitudes contracts the tail network with
                                v_head as one more leaf, once, in complex128, giving
                                A[s2] = sum_c T_tail[s2, c] v_head[c] without forming
                                T_tail.  Needs tree = NULL and planner-chosen slicing
                                (TN_EINVAL otherwise).  0 = one tree whose root gives A. */
    int32_t restarts;        /* randomised greedy trees tried (>= 1) */
    int32_t cost_model;      /* 0 = FLOP/byte roofline model, 1 = learned MLP */
    uint64_t seed;
    int64_t max_workspace_bytes;  /* cap for the per-launch workspace (0 = 32 GiB) */
    const struct tn_mlp_s* model; /* trained step-time model for cost_model = 1 (NULL = FLOP model) */
    int32_t slicing;         /* planner-chosen slicing (appendix A, "Dynamic slicing"):
                                2 = dynamic: edges are sliced one at a time, each the
                                greedy choice on the current tree, and the tree is
                                re-tuned by subtree reconfiguration after every sliced
                                edge; 1 = one-shot: greedy slicing of the whole set on
                                the unsliced tree, then one re-tune and a top-up;
                                0 = both, per candidate tree, keeping the one with less
                                total work over all slices */
} tn_plan_opts;

typedef struct {
    uint64_t n_slices;            /* 2^n_sliced */
    int32_t n_sliced;             /* sliced edges */
    int32_t batch_log2;           /* slices per launch sequence (log2) */
    int32_t n_open, n_leaves, n_steps;
    int32_t n_c;                  /* cut legs between head and tail (bighead), else 0 */
    int32_t max_log2_size;        /* largest intermediate of one slice (log2 elements) */
    int32_t acc_log2;             /* accumulator length = 2^acc_log2 complex128 */
    double cmacs_per_slice;       /* complex multiply-adds per slice, executed tree */
    double cmacs_per_slice_unmerged; /* same before branch merging */
    double cmacs_invariant;       /* slice-invariant work done once per plan */
    double cmacs_tail;            /* tail network with the v_head leaf, per tn_amplitudes call (bighead) */
    double bytes_per_slice;       /* algorithmic HBM bytes per slice (operands + results) */
    double cmacs_per_batch;       /* complex multiply-adds per launch sequence */
    double bytes_per_batch;
    uint64_t workspace_bytes;     /* minimum ws_bytes for tn_contract_slices */
    uint64_t tail_workspace_bytes;/* minimum ws_bytes for tn_amplitudes (bighead; else 0) */
    int32_t n_dense_steps;        /* steps run on MFMA (tiled, skinny or panel) */
    int32_t n_small_steps;        /* steps run on the VALU kernels (tile, split-K, streaming) */
    int32_t cost_model_used;      /* 0 FLOP count, 1 learned model, 2 learned model asked but
                                     outside its training support (FLOP count used) */
    int32_t n_candidates;         /* candidate trees/slicings ranked */
    double predicted_ms;          /* learned model's predicted time of the whole job (0 if unused) */
    uint64_t graph_replays;       /* launch groups replayed from captured graphs on this plan so far */
    uint64_t graph_launches;      /* graph launches that replayed them (up to 16 groups per launch) */
    int32_t lanes;                /* concurrent lanes of launch groups (tn_plan_set_lanes) */
    uint64_t lanes_workspace_bytes; /* ws_bytes for tn_contract_slices to use every lane */
} tn_plan_stats;

typedef struct {
    double F_unif;     /* Eq. (1) over all 2^n2 amplitudes, equal weights */
    double F_self;     /* 2^n * sum P^2 / sum P - 1 */
    double P_s1;       /* marginal probability sum_s2 P(s1; s2) */
    double cond_xeb;   /* XEB of P(s2|s1) over the open qubits (0 up to rounding) */
    double p_max, p_min;
} tn_xeb_result;

/* Build a plan (host only; no device work).  Section "The algorithm" and
 * appendix A: contraction order (randomised greedy, or the caller's tree),
 * slicing to the memory target, slice-invariant subtrees hoisted, branch
 * merging, per-step layouts; optionally the big-head split (opts->bighead).
 *   c              circuit (copied)
 *   open_q/fixed_q disjoint, together every qubit exactly once
 *   fixed_bits     s1, one byte (0/1) per fixed qubit, in fixed_q order
 *   tree           NULL = planner's order; else SSA pairs over the leaves
 *   sliced         NULL with n_sliced = -1: planner chooses; else the edges to
 *                  slice (must be internal edges, not open legs)
 *   opts           NULL = defaults (C64, target 2^30, planner batching)
 * Errors: TN_EINVAL for a bad circuit, overlapping or missing qubits, a bad
 * tree or edge; TN_ENOMEM.  On success *out owns every input it needs. */
tn_status tn_plan(const tn_circuit* c,
                  const int32_t* open_q, int32_t n_open,
                  const int32_t* fixed_q, const uint8_t* fixed_bits, int32_t n_fixed,
                  const tn_tree* tree, const tn_edge* sliced, int32_t n_sliced,
                  const tn_plan_opts* opts, tn_plan_t* out);

/* Statistics of a plan (host only). */
tn_status tn_plan_stats_get(tn_plan_t p, tn_plan_stats* out);

/* The sliced edges in slice-bit order; *n receives the count (<= cap are
 * written). */
tn_status tn_plan_sliced_edges(tn_plan_t p, tn_edge* out, int32_t cap, int32_t* n);

/* JSON description of the plan (tree, leaves' edge names, sliced and batch
 * edges, per-step shapes, costs and kernel choices).  Writes at most cap
 * bytes including the terminating NUL; *need receives the full size. */
tn_status tn_plan_export_json(tn_plan_t p, char* buf, size_t cap, size_t* need);

/* Contract slices [slice_begin, slice_end) and add their sum, in float64, to
 * the accumulator d_acc (2^acc_log2 complex128, caller-zeroed before the
 * first call).  Section "The algorithm": slicing turns the network into
 * independent subtasks, one per assignment of the sliced edges, whose results
 * add up to the unsliced result; appendix B ("Computation details") sums the
 * final tensors of the subtasks.  Slice j fixes the i-th sliced edge to bit
 * i of j.  Sums over disjoint ranges add up to the sum over their union.
 * Runs of at least two full launch groups (2^batch_log2 slices each) replay
 * one captured HIP graph; other groups, and every group while per-step
 * profiling is on, are launched one kernel at a time (same kernels, bitwise
 * equal results).  d_workspace must hold stats.workspace_bytes (with
 * lanes, see tn_plan_set_lanes).  The first call on a device uploads the
 * plan's leaves and computes its slice-invariant subtrees.  Asynchronous on
 * hip_stream.
 * Errors: TN_EINVAL (range, sizes, NULL), TN_EDEVICE. */
tn_status tn_contract_slices(tn_plan_t p, void* d_workspace, size_t ws_bytes,
                             double* d_acc, uint64_t slice_begin, uint64_t slice_end,
                             void* hip_stream);

/* Same for an explicit host list of slice ids (each < n_slices). */
tn_status tn_contract_slice_list(tn_plan_t p, void* d_workspace, size_t ws_bytes,
                                 double* d_acc, const uint64_t* h_slice_ids, uint64_t n_ids,
                                 void* hip_stream);

/* Turn the accumulator into the 2^n_open amplitudes d_amps (complex128):
 * with the big-head split this contracts the tail with the summed head
 * vector (section "Big-head simulation", the final inner product
 * v_head . v_tail(s2)): the accumulator is copied to the host, placed as the
 * tail's last leaf and the tail contracted on hip_stream, which is
 * synchronised (the tail's slice-free steps run at the first call only).
 * Cost of the split form: two stream synchronisations and a round trip of
 * 2^n_c complex128 through host memory (16 MiB for a 20-leg cut), once per
 * job, not per slice.  Without the split the accumulator already holds A and
 * is copied on the device (asynchronous).
 * d_workspace must hold stats.tail_workspace_bytes (TN_EINVAL otherwise). */
tn_status tn_amplitudes(tn_plan_t p, const double* d_acc, double* d_amps,
                        void* d_workspace, size_t ws_bytes, void* hip_stream);

/* Statistics of d_amps (2^n_open complex128) in float64 on the device:
 * Eq. (1) with equal weights, F_self, P(s1) and the conditional XEB
 * (appendix C).  `weight` multiplies every probability first (1 for full
 * amplitudes; 2^k / |S| for partial sums over a sample S of slices).  If
 * n_ks > 0, h_topk[i] receives the XEB of the ks[i] largest probabilities
 * (post-selection curve of section "Fidelity").  Synchronises the stream.
 * TN_EINVAL for NULL pointers, n_open outside [0, 40], n_qubits below
 * n_open or above 1023 (2^n_qubits must be a finite double), a
 * non-positive weight or a top-k size outside [1, 2^n_open]. */
tn_status tn_xeb(const double* d_amps, int32_t n_open, int32_t n_qubits, double weight,
                 const int64_t* ks, int32_t n_ks, double* h_topk,
                 tn_xeb_result* out, void* hip_stream);

/* Sampling from the conditional distribution of the open qubits (appendix C
 * defines P(s2 | s1) = P(s1; s2) / P(s1); the conclusion notes that the
 * method can sample from it): draws n_samples indices s2 (open-qubit
 * bitstrings, first open qubit the most significant bit, as in d_amps) by
 * inverse transform.  Sample i is the smallest s2 with
 * cdf[s2] > d_uniform[i] * cdf[2^n_open - 1], cdf the float64 inclusive
 * prefix sum of |A[s2]|^2 in index order (summed in a fixed order: results
 * are bitwise repeatable); if every amplitude is zero, every sample is
 * 2^n_open - 1.  d_amps: 2^n_open complex128; d_uniform: n_samples doubles
 * in [0, 1), drawn by the caller; d_out: n_samples uint64; all device
 * memory owned by the caller.  d_workspace must hold
 * tn_sample_workspace_bytes(n_open) bytes.  Asynchronous on hip_stream.
 * TN_EINVAL for NULL pointers (d_uniform and d_out may be NULL when
 * n_samples is 0), n_open outside [0, 34] or a small workspace. */
size_t tn_sample_workspace_bytes(int32_t n_open);
tn_status tn_sample(const double* d_amps, int32_t n_open, const double* d_uniform, uint64_t n_samples,
                    uint64_t* d_out, void* d_workspace, size_t ws_bytes, void* hip_stream);

/* tn_sample without a workspace argument and without any allocation, for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, same
 * kernels and bitwise the same samples as tn_sample.  The workspace is a
 * file-scope device array of 8.0 MiB (2^20 probabilities and their scan
 * levels) that every GPU the library runs on holds until the process ends;
 * its address on a device is looked up once, at the first call on that
 * device.  Every call on a GPU shares that GPU's array: calls that overlap
 * on one GPU (other streams, other threads) race and must be serialised by
 * the caller.  Nothing in the array needs clearing between calls (every
 * element read is first written by the same call).  Asynchronous on
 * hip_stream.  TN_EINVAL for NULL pointers (d_uniform and d_out may be NULL
 * when n_samples is 0) or n_open outside [0, 20]; TN_EDEVICE for launch
 * errors. */
tn_status tn_sample_noalloc(const double* d_amps, int32_t n_open, const double* d_uniform, uint64_t n_samples,
                            uint64_t* d_out, void* hip_stream);

/* Mixing the most probable computed bitstrings with random ones (section
 * "Discussions", footnote: the k bitstrings of highest probability are mixed
 * with many random bitstrings, which removes most of the correlation of the
 * set while its XEB stays positive).  d_amps: 2^n_open complex128 amplitudes
 * of the open qubits (first open qubit the most significant bit), open_q
 * ascending; open_q and fixed_q together are the qubits 0..n_qubits-1, and
 * fixed_bits (one byte per fixed qubit) is s1.  Writes d_out[0, k): the k
 * indices of largest |A|^2 (computed as re*re + im*im, each product rounded;
 * ties at the threshold go to the lower index), in increasing index order,
 * as whole n-bit strings with qubit q at bit n_qubits-1-q; and
 * d_out[k, k + n_random): the caller's uniform random 64-bit words
 * d_random_words masked to n_qubits bits.  out receives P_top (sum of the
 * selected probabilities, in a fixed order), F_top = 2^n / k * P_top - 1
 * (the XEB of the top k alone) and F_mix_expected = (2^n P_top + n_random) /
 * (k + n_random) - 1, the XEB of the whole set in expectation over the random
 * strings (a uniform random string has expected 2^n P = 1).  Device buffers
 * are caller-owned; d_workspace holds tn_mix_workspace_bytes(n_open) bytes.
 * Synchronises the stream.  TN_EINVAL for NULL pointers, qubit lists that do
 * not partition 0..n-1, n_qubits > 64, n_open > 34, k > 2^n_open or a small
 * workspace. */
typedef struct {
    double P_top, F_top, F_mix_expected;
} tn_mix_result;
size_t tn_mix_workspace_bytes(int32_t n_open);
tn_status tn_mix_topk(const double* d_amps, int32_t n_qubits, const int32_t* open_q, int32_t n_open,
                      const int32_t* fixed_q, const uint8_t* fixed_bits, int32_t n_fixed, uint64_t k,
                      const uint64_t* d_random_words, uint64_t n_random, uint64_t* d_out, void* d_workspace,
                      size_t ws_bytes, tn_mix_result* out, void* hip_stream);

/* Per-step timing of the slice-dependent steps, for measurement and for the
 * learned step-time model.  While enabled, tn_contract_slices records HIP
 * events around every step it launches (two event sets used alternately, so
 * the host never waits on the group it has just queued) and accumulates the
 * elapsed times. */
typedef struct {
    int32_t m_log, n_log, k_log, b_log;   /* step shape C[b,m,n] = sum_k A[k,b,m] B[k,b,n] */
    int32_t kernel, tile;                 /* 0 VALU tile, 1 MFMA tile, 2 split-K, 3 VALU streaming,
                                             4 skinny MFMA, 5 panel MFMA; tile id */
    double cmacs;                         /* complex multiply-adds per launch */
    double bytes;                         /* algorithmic bytes per launch (A + B + C) */
    double total_ms;                      /* summed GPU time of this step's launches */
    uint64_t launches;
    char kernel_name[48];                 /* device function name as profilers show it */
} tn_step_profile;

/* Run later tn_contract_slices calls on `lanes` concurrent HIP streams
 * (1 .. 8; default 1).  Section "The algorithm": the subtasks of a sliced
 * network are independent, so runs of launch groups can execute at once; two
 * lanes let one lane's bandwidth-bound steps overlap another's
 * compute-bound ones.  A call with at least two full launch groups per lane
 * splits its groups into contiguous runs, one per lane: lane 0 runs on the
 * caller's stream with the caller's accumulator and workspace, lane i on a
 * private stream (default priority) at d_workspace + i * stride (stride =
 * stats.workspace_bytes rounded up to 256 bytes) with a private float64
 * accumulator; the caller's stream then waits for every lane and adds the
 * lanes' sums in lane order, so results are deterministic for a given lane
 * count and equal to the one-lane result up to float64 rounding of the
 * order of the additions.  A call uses as many lanes as whole workspaces fit
 * in ws_bytes (stats.lanes_workspace_bytes fits all); step timing, slice
 * lists and short ranges use one lane.  Each extra lane allocates, on its
 * first use, its stream, 2^acc_log2 complex128 and a few bytes of device
 * memory, and captures its own graphs; lowering the count releases the
 * extra lanes after their work has finished.  Errors: TN_EINVAL (range),
 * TN_EDEVICE. */
tn_status tn_plan_set_lanes(tn_plan_t p, int32_t lanes);

/* Enable (1) or disable (0) step timing; enabling resets the counters. */
tn_status tn_plan_set_profiling(tn_plan_t p, int32_t enable);

/* Read the counters (synchronises outstanding timed work).  Entry i is the
 * i-th slice-dependent step in execution order; the last entry is the float64
 * slice sum.  *n receives the number of entries (<= cap are written). */
tn_status tn_plan_step_profile(tn_plan_t p, tn_step_profile* out, int32_t cap, int32_t* n);

/* Autotuner: for every distinct slice-dependent step shape (m, n, k, batch,
 * precision) time each candidate kernel tile on the data of one real launch
 * group (HIP events, median of `reps` launches after one warm-up) and keep
 * the fastest.  Choices are cached in the text file `cache_path` (NULL = no
 * cache), keyed by GPU architecture, shape and precision; cached shapes are
 * not re-timed.  The accumulator is used as scratch and must be re-zeroed by
 * the caller afterwards.  Returns the number of shapes timed in *n_tuned. */
tn_status tn_plan_autotune(tn_plan_t p, void* d_workspace, size_t ws_bytes, double* d_acc_scratch,
                           const char* cache_path, int32_t reps, int32_t* n_tuned, void* hip_stream);

/* Open qubits read off a contraction order (section "Big-head simulation of
 * quantum circuits": the order is found first and the open qubits are chosen
 * from it).  The network with every qubit closed is planned with `opts`
 * (NULL = defaults); a qubit ends at its last two-qubit gate, or at its own
 * node if it has none.  Among the tree's nodes with at most half of the
 * leaves under them whose subtree holds the ends of at least n_open qubits,
 * the one with the fewest legs to the rest of the network (ties: the fewest
 * leaves) is the tail (the whole network if there is none); the n_open lowest-id qubits
 * ending under it are written to h_open (ascending; caller-owned host array
 * of n_open) and its leg count, the head-tail cut when exactly these qubits
 * are opened, to *n_cut.  Host only.  TN_EINVAL for a bad circuit, NULL
 * pointers or n_open outside [1, min(n_qubits, 40)]. */
tn_status tn_choose_open_qubits(const tn_circuit* c, int32_t n_open, const tn_plan_opts* opts, int32_t* h_open,
                                int32_t* n_cut);

/* Kernel configurations that can run step `step` (index into the plan's
 * steps in execution order, as listed by tn_plan_export_json): up to cap
 * (kernel, tile) pairs are written to h_kernels / h_tiles (host arrays owned
 * by the caller), their number to *n.  Split-K is offered only while the
 * step uses it. */
tn_status tn_plan_step_candidates(tn_plan_t p, int32_t step, int32_t* h_kernels, int32_t* h_tiles,
                                  int32_t cap, int32_t* n);

/* Run step `step` with one of its candidate configurations from now on
 * (overrides the planner's or the autotuner's choice; a captured graph is
 * rebuilt at the next launch).  A slice-invariant step already computed on
 * the device keeps its result.  TN_EINVAL if (kernel, tile) is not a
 * candidate; TN_ESTATE while step timing is enabled. */
tn_status tn_plan_set_step_kernel(tn_plan_t p, int32_t step, int32_t kernel, int32_t tile);

/* ---- learned step-time model ------------------------------------------
 * A 3-layer perceptron d_in -> hidden -> hidden -> 1 (ReLU) on the device,
 * FP32, that maps step features to log(step milliseconds).  Forward,
 * backward and Adam run in the library's own kernels.  Parameters are one
 * flat array: W1 (d_in x hidden, row-major), b1, W2 (hidden x hidden), b2,
 * W3 (hidden x 1), b3.  Not from the paper, whose cost is the FLOP count
 * 2^(nA+nB+nAB) of appendix A (Fig. 3); that count stays the fallback. */
typedef struct tn_mlp_s* tn_mlp_t;

#define TN_STEP_FEATURES 12

/* Features of one step (shape logs, operand and output logs, log work, log
 * bytes at the plan's storage width, kernel class flags: MFMA, VALU tile,
 * split-K; the streaming kernel has none set), written to
 * out[TN_STEP_FEATURES]. */
tn_status tn_step_features(int32_t m_log, int32_t n_log, int32_t k_log, int32_t b_log, int32_t kernel,
                           tn_precision prec, float* out);

/* Features of a plan's slice-dependent steps in execution order (the order of
 * tn_plan_step_profile); h_out holds cap_steps * TN_STEP_FEATURES floats. */
tn_status tn_plan_step_features(tn_plan_t p, float* h_out, int32_t cap_steps, int32_t* n_steps);

/* Create a model on the current device with He-normal weights from `seed`. */
tn_status tn_mlp_create(int32_t d_in, int32_t hidden, uint64_t seed, tn_mlp_t* out);
tn_status tn_mlp_num_params(tn_mlp_t m, int64_t* n);
tn_status tn_mlp_get_params(tn_mlp_t m, float* h_params, int64_t n);
tn_status tn_mlp_set_params(tn_mlp_t m, const float* h_params, int64_t n);

/* d_y[batch] = model(d_x[batch x d_in]) (device pointers). */
tn_status tn_mlp_forward(tn_mlp_t m, const float* d_x, int32_t batch, float* d_y, void* hip_stream);

/* Gradient of mean((model(x) - t)^2) with respect to every parameter,
 * copied to h_grads (n_params floats, may be NULL); loss to *h_loss (may be
 * NULL).  Synchronises the stream. */
tn_status tn_mlp_gradient(tn_mlp_t m, const float* d_x, const float* d_t, int32_t batch, float* h_grads,
                          float* h_loss, void* hip_stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on that gradient. */
tn_status tn_mlp_train_step(tn_mlp_t m, const float* d_x, const float* d_t, int32_t batch, float lr,
                            float* h_loss, void* hip_stream);

/* Feature box seen in training: a plan whose steps leave it (by more than
 * `margin` per feature) is ranked by the FLOP count instead. */
tn_status tn_mlp_set_support(tn_mlp_t m, const float* h_min, const float* h_max, int32_t n_feat, float margin);

void tn_mlp_destroy(tn_mlp_t m);

/* Release a plan and its device memory (NULL is ignored). */
void tn_plan_destroy(tn_plan_t p);

/* Message of the last failure on this thread ("" if none). */
const char* tn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TN_H */
