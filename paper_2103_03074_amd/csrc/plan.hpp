// Host-side planner of the sliced big-head contraction.
//
// Builds the circuit's tensor network (single-qubit gates absorbed into
// two-qubit gates; section "Computing bitstring probabilities"), finds a
// pairwise contraction order, slices edges until every intermediate of one
// slice fits the memory target (appendix A, "Dynamic slicing"), hoists
// slice-invariant subtrees, optionally splits head and tail (section
// "Big-head simulation"), merges small branches (appendix B, "GPU
// efficiency") and assigns each tensor a memory layout so that every step
// reads its operands as plain strided arrays.
#pragma once

#include <complex>
#include <cstdint>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "../../include/tn.h"

namespace tn {

using cd = std::complex<double>;

struct EdgeName {
    int q, t;
    bool operator<(const EdgeName& o) const { return q < o.q || (q == o.q && t < o.t); }
    bool operator==(const EdgeName& o) const { return q == o.q && t == o.t; }
};

// A dense tensor whose i-th leg is address bit i.
struct HostTensor {
    std::vector<int> legs;
    std::vector<cd> data;
};

struct Network {
    int n_qubits = 0;
    std::vector<EdgeName> edge_name;          // edge id -> (q, t)
    std::vector<int> end0, end1;              // leaves holding the edge (end1 = -1: open leg)
    std::vector<HostTensor> leaves;
    std::vector<int> open_edges;              // output order, index 0 = most significant bit
    int find_edge(int q, int t) const;
};

// Canonical network of a circuit; returns an error message or "".
std::string build_network(const tn_circuit& c, const std::vector<int>& open_q,
                          const std::vector<int>& fixed_q, const std::vector<uint8_t>& bits,
                          Network& out);

// Sorted small integer sets.
using Legs = std::vector<int>;
Legs set_union(const Legs& a, const Legs& b);
Legs set_inter(const Legs& a, const Legs& b);
Legs set_minus(const Legs& a, const Legs& b);
Legs set_xor(const Legs& a, const Legs& b);

struct Tree {
    int n_leaves = 0;
    std::vector<int> lhs, rhs;   // step s creates node n_leaves + s
    int n_nodes() const { return n_leaves + (int)lhs.size(); }
    int root() const { return n_nodes() - 1; }
};

// Randomised greedy order over the given leaves' legs.
Tree greedy_tree(const std::vector<Legs>& leaf_legs, uint64_t seed, double alpha, double temperature);

// Order from recursive min-cut bisection (leaf groups of <= leaf_size tensors
// contracted greedily); eps is the allowed size imbalance of each bisection.
// time_cap / space_cap (log2; 0 = none): every bisection's own contraction
// (the two parts joined) should stay within 2^time_cap multiply-adds and a
// 2^space_cap output; bisections over a cap are retried with other seeds
// and imbalances, keeping the one closest to the caps.
Tree partition_tree(const std::vector<Legs>& leaf_legs, uint64_t seed, double eps, int leaf_size,
                    int open_w, int time_cap = 0, int space_cap = 0);

// Subtree reconfiguration: repeatedly replace subtrees of up to max_frontier
// frontier tensors by their optimal order (cost per slice with the edges in
// in_s removed, intermediates above 2^target penalised).
// objective 0: complex multiply-adds; 1: roofline time estimate (branch
// merging) with dense_rate the flop rate of MFMA-shaped steps and each
// step's output bytes counted write_weight times.
Tree reconfigure(const std::vector<Legs>& leaf_legs, const Tree& in, const std::vector<char>& in_s, int target,
                 int max_frontier, int passes, int objective = 0, int esize = 8, double dense_rate = 110e12,
                 double write_weight = 1.0);
// Roofline time estimate of a tree (same units as objective 1).
double tree_time_estimate(const std::vector<Legs>& leaf_legs, const Tree& t, const std::vector<char>& in_s, int esize,
                          double dense_rate = 110e12, double write_weight = 1.0);
// Measured flop rate (Eq. (3) flops per second) of MFMA-shaped steps per
// precision on MI355X, for the time objective.
double dense_step_rate(tn_precision prec);
// Weight of output bytes against input bytes in the time objective, per
// precision (measured on the 40-qubit workload).
double write_weight(tn_precision prec);

// Leaves contracted one after another in network (time) order.
Tree time_order_tree(int n_leaves);

// Kernel classes a step can run on.
enum StepKernel : int32_t { K_SMALL = 0, K_MFMA = 1, K_SPLITK = 2, K_STREAM = 3, K_SKINNY = 4, K_PANEL = 5 };

// One pairwise step as executed: C[b, m, n] = sum_k A[k, b, m] * B[k, b, n].
// A is stored [K legs | batch legs | M legs] from the most to the least
// significant bit, B likewise with N, so both are plain strided arrays; C is
// stored in the layout its consumer wants (c_pos_* give the address bit of
// each logical bit).
struct Step {
    int node;                 // tree node produced
    int a_node, b_node;       // operands (A = the side with M legs)
    int m_log, n_log, k_log, b_log;
    std::vector<int> c_pos_m, c_pos_n, c_pos_b;
    bool invariant;           // slice-invariant: computed once per plan
    int kernel;               // StepKernel
    int tile;                 // tile configuration id for the kernel
    int splitk_log;           // K split into 2^splitk_log parts (K_SPLITK)
    double cmacs;             // 2^(m+n+k+b)
    double bytes;             // algorithmic bytes at the storage width
    uint64_t c_off;           // offset of C in its arena (workspace or plan memory)
    uint64_t scratch_off;     // split-K partials (workspace)
    uint64_t conv_off = ~uint64_t(0);   // split A planes of a mixed-precision panel step, or ~0
};

// Where a node's tensor lives when it is read.
enum NodeHome : int32_t { HOME_LEAF = 0, HOME_PLAN = 1, HOME_WS = 2 };

struct NodeInfo {
    Legs legs;                // legs with sliced (non-batch) edges removed, batch legs kept
    std::vector<int> layout;  // leg at each address bit (bit 0 first)
    std::vector<int> sliced_bits;  // leaves: slice-bit index of each outer-sliced leg on top
    bool dep = false;         // depends on the slice id
    int home = HOME_WS;
    int slot = 0;             // index of this tensor's max-magnitude slot (low-precision scaling)
    uint64_t off = 0;         // offset in its arena (elements)
    int parent = -1;
};

struct Plan {
    Network net;
    Tree tree;
    tn_plan_opts opts{};
    std::vector<int> sliced;        // edge ids, slice bit i = sliced[i]
    std::vector<int> batch;         // the first batch_log2 sliced edges are batch legs
    int batch_log2 = 0;
    std::vector<NodeInfo> nodes;
    std::vector<Step> steps;        // execution order: invariant steps first
    std::vector<int> step_of_node;  // node -> index in steps (-1 for leaves)
    int n_invariant_steps = 0;
    int esize = 8;                  // bytes per complex element of the storage
    uint64_t ws_elems = 0;          // per-batch workspace (elements), incl. split-K scratch
    uint64_t plan_elems = 0;        // plan-owned device memory (leaves + invariants)
    int root_log2 = 0;              // result legs of the root (without batch legs)
    int n_static_slots = 0;         // slots of leaves and invariant tensors come first
    tn_plan_stats stats{};
    double unmerged_cmacs_per_slice = 0;
    // big-head split: this plan is the head (its open legs are the cut legs
    // c, its accumulator v_head[c]); `tail` is the tail network plus one leaf
    // that receives v_head (the last leaf, forced slice-dependent) and whose
    // root is A[s2]
    std::shared_ptr<Plan> tail;
    std::vector<int> full_open;     // open legs of the whole network (amplitude index)
    std::vector<char> force_dep;    // leaves treated as slice-dependent (their data arrives later)
};

// Learned step-time model as seen by the planner: predict log(ms) of each
// step from its features, and say whether a feature row is inside the
// training support.
struct CostModel {
    std::function<std::string(const std::vector<float>& feats, int n_rows, std::vector<float>& log_ms)> predict;
    std::function<bool(const float* row)> in_support;
};

// Full planning pipeline.
std::string make_plan(const tn_circuit& c, const std::vector<int>& open_q,
                      const std::vector<int>& fixed_q, const std::vector<uint8_t>& bits,
                      const tn_tree* tree, const tn_edge* sliced, int n_sliced,
                      const tn_plan_opts& opts, Plan& out, const CostModel* cm = nullptr);

// Open qubits chosen from a contraction order of the closed network (the
// qubits ending under the node with the fewest legs that holds n_open
// qubit ends); cut_out receives that node's leg count.
std::string choose_open_qubits(const tn_circuit& c, int n_open, const tn_plan_opts& opts, std::vector<int>& open_out,
                               int& cut_out);


void step_features(int m, int n, int k, int b, int kernel, int esize, float* out);
constexpr int kStepFeatures = 12;

std::string plan_to_json(const Plan& p);

// Cost of a tree with a set of sliced edges (no batching).
struct SliceCost {
    double per_slice = 0;     // complex MACs of slice-dependent steps
    double invariant = 0;     // complex MACs of slice-invariant steps
    int max_log2 = 0;         // largest intermediate of a slice (log2 elements)
    double total(int k) const { return per_slice * (double)(1ULL << k) + invariant; }
};
SliceCost slice_cost(const Network& net, const Tree& t, const std::vector<char>& in_s);

tn_plan_opts default_opts();

}  // namespace tn
