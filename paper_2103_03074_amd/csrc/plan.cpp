// Contraction order, slicing, batching, layouts and the step list (host).
//
// Paper passages followed:
//  - pairwise cost 2^(nA + nB + nAB) for bond dimension 2 (appendix A, Fig. 3);
//  - greedy contraction order inside sub-graphs (section "The algorithm");
//  - slicing: fix n_e edges, enumerate the 2^n_e subtasks and sum
//    (section "The algorithm", appendix A "Dynamic slicing");
//  - the head/tail split with the head vector reused for every s2
//    (section "Big-head simulation of quantum circuits").
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <numeric>
#include <queue>
#include <random>
#include <set>
#include <sstream>
#include <cstdio>
#include <cstdlib>

#include "plan.hpp"
#include "tiles.hpp"

namespace tn {

Legs set_union(const Legs& a, const Legs& b) {
    Legs r;
    std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(r));
    return r;
}
Legs set_inter(const Legs& a, const Legs& b) {
    Legs r;
    std::set_intersection(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(r));
    return r;
}
Legs set_minus(const Legs& a, const Legs& b) {
    Legs r;
    std::set_difference(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(r));
    return r;
}
Legs set_xor(const Legs& a, const Legs& b) {
    Legs r;
    std::set_symmetric_difference(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(r));
    return r;
}

tn_plan_opts default_opts() {
    tn_plan_opts o{};
    o.prec = TN_C64;
    o.max_log2_size = 30;
    o.n_slice_edges = -1;
    o.batch_log2 = -1;
    o.branch_merge = 0;
    o.bighead = 0;
    o.restarts = 8;
    o.cost_model = 0;
    o.seed = 0;
    o.max_workspace_bytes = 0;
    o.model = nullptr;
    o.slicing = 0;
    return o;
}

// ---------------------------------------------------------------- greedy

Tree greedy_tree(const std::vector<Legs>& leaf_legs, uint64_t seed, double alpha, double temperature) {
    const int L = (int)leaf_legs.size();
    int n_edges = 0;
    for (auto& l : leaf_legs)
        for (int e : l) n_edges = std::max(n_edges, e + 1);
    std::vector<Legs> legs(leaf_legs);
    legs.reserve(2 * L);
    std::vector<char> alive(L, 1);
    std::vector<std::array<int, 2>> owner(n_edges, {-1, -1});
    for (int i = 0; i < L; ++i)
        for (int e : legs[i]) {
            if (owner[e][0] < 0) owner[e][0] = i;
            else owner[e][1] = i;
        }
    std::mt19937_64 rng(seed * 0x9E3779B97F4A7C15ULL + 12345);
    std::uniform_real_distribution<double> unif(1e-300, 1.0);
    struct Cand {
        double s;
        int a, b;
        bool operator<(const Cand& o) const {
            if (s != o.s) return s > o.s;
            if (a != o.a) return a > o.a;
            return b > o.b;
        }
    };
    std::priority_queue<Cand> pq;
    auto score = [&](int a, int b) {
        size_t la = legs[a].size(), lb = legs[b].size();
        size_t shared = set_inter(legs[a], legs[b]).size();
        size_t lc = la + lb - 2 * shared;
        double raw = std::exp2((double)lc) - alpha * (std::exp2((double)la) + std::exp2((double)lb));
        double s = raw >= 0 ? std::log2(1.0 + raw) : -std::log2(1.0 - raw);
        if (temperature > 0) s -= temperature * (-std::log(-std::log(unif(rng))));
        return s;
    };
    auto push = [&](int a, int b) {
        if (a > b) std::swap(a, b);
        pq.push({score(a, b), a, b});
    };
    {
        std::set<std::pair<int, int>> seen;
        for (int e = 0; e < n_edges; ++e) {
            int a = owner[e][0], b = owner[e][1];
            if (a < 0 || b < 0 || a == b) continue;
            if (seen.insert({std::min(a, b), std::max(a, b)}).second) push(a, b);
        }
    }
    Tree t;
    t.n_leaves = L;
    int n_alive = L;
    while (n_alive > 1) {
        int a = -1, b = -1;
        while (!pq.empty()) {
            Cand c = pq.top();
            pq.pop();
            if (alive[c.a] && alive[c.b]) {
                a = c.a;
                b = c.b;
                break;
            }
        }
        if (a < 0) {   // disconnected pieces: join the two smallest
            std::vector<int> ids;
            for (int i = 0; i < (int)alive.size(); ++i)
                if (alive[i]) ids.push_back(i);
            std::sort(ids.begin(), ids.end(), [&](int x, int y) {
                return legs[x].size() != legs[y].size() ? legs[x].size() < legs[y].size() : x < y;
            });
            a = std::min(ids[0], ids[1]);
            b = std::max(ids[0], ids[1]);
        }
        const int c = (int)legs.size();
        legs.push_back(set_xor(legs[a], legs[b]));
        for (int e : set_inter(legs[a], legs[b])) owner[e] = {-1, -1};
        alive[a] = alive[b] = 0;
        alive.push_back(1);
        --n_alive;
        t.lhs.push_back(a);
        t.rhs.push_back(b);
        std::set<int> nbs;
        for (int e : legs[c]) {
            for (int s = 0; s < 2; ++s)
                if (owner[e][s] == a || owner[e][s] == b) owner[e][s] = c;
            int other = owner[e][0] == c ? owner[e][1] : owner[e][0];
            if (other >= 0 && other != c) nbs.insert(other);
        }
        for (int nb : nbs) push(c, nb);
    }
    return t;
}

// ------------------------------------------------------------ tree legs

namespace {

struct TreeLegs {
    std::vector<Legs> node;   // legs of each node (no slicing)
    std::vector<Legs> uni;    // per step: legs(a) U legs(b)
    std::vector<int> parent;
};

TreeLegs tree_legs(const Network& net, const Tree& t) {
    TreeLegs tl;
    tl.node.resize(t.n_nodes());
    tl.parent.assign(t.n_nodes(), -1);
    for (int i = 0; i < t.n_leaves; ++i) {
        tl.node[i] = net.leaves[i].legs;
        std::sort(tl.node[i].begin(), tl.node[i].end());
    }
    tl.uni.resize(t.lhs.size());
    for (size_t s = 0; s < t.lhs.size(); ++s) {
        int a = t.lhs[s], b = t.rhs[s], c = t.n_leaves + (int)s;
        tl.node[c] = set_xor(tl.node[a], tl.node[b]);
        tl.uni[s] = set_union(tl.node[a], tl.node[b]);
        tl.parent[a] = tl.parent[b] = c;
    }
    return tl;
}

int count_not_in(const Legs& l, const std::vector<char>& in_s) {
    int c = 0;
    for (int e : l) c += !in_s[e];
    return c;
}

SliceCost slice_cost_tl(const TreeLegs& tl, const Tree& t, const std::vector<char>& in_s) {
    SliceCost sc;
    std::vector<char> dep(t.n_nodes(), 0);
    for (int i = 0; i < t.n_leaves; ++i)
        for (int e : tl.node[i]) dep[i] |= in_s[e];
    for (size_t s = 0; s < t.lhs.size(); ++s) {
        int c = t.n_leaves + (int)s;
        dep[c] = dep[t.lhs[s]] | dep[t.rhs[s]];
        double w = std::exp2((double)count_not_in(tl.uni[s], in_s));
        if (dep[c]) sc.per_slice += w;
        else sc.invariant += w;
        sc.max_log2 = std::max(sc.max_log2, count_not_in(tl.node[c], in_s));
    }
    return sc;
}

// Greedy slicing: repeatedly fix the edge whose removal gives the lowest total
// work, among the legs of the largest intermediates, until the memory target
// and the requested count are both met.
// One greedy slicing choice on the current tree: among the legs of the
// largest tensors (those at the largest size while over the target, else
// within a factor 2 of it), the edge whose slicing gives the lowest total
// cost over all slices; -1 if there is none.
static int greedy_slice_step(const Network& net, const Tree& t, const TreeLegs& tl, std::vector<char>& in_s,
                             const std::vector<char>& is_open, int k, bool over) {
    const SliceCost cur = slice_cost_tl(tl, t, in_s);
    const int thresh = over ? cur.max_log2 : std::max(0, cur.max_log2 - 1);
    std::set<int> cands;
    for (int c = t.n_leaves; c < t.n_nodes(); ++c) {
        if (count_not_in(tl.node[c], in_s) < thresh) continue;
        for (int e : tl.node[c])
            if (!in_s[e] && !is_open[e]) cands.insert(e);
    }
    int best = -1;
    double best_cost = 0;
    for (int e : cands) {
        in_s[e] = 1;
        SliceCost nc = slice_cost_tl(tl, t, in_s);
        in_s[e] = 0;
        double tot = nc.total(k + 1);
        if (best < 0 || tot < best_cost * (1 - 1e-12)) {
            best = e;
            best_cost = tot;
        }
    }
    return best;
}

std::vector<int> greedy_slice(const Network& net, const Tree& t, const TreeLegs& tl, int target,
                              int n_force, std::vector<int> sliced) {
    const int E = (int)net.edge_name.size();
    std::vector<char> is_open(E, 0), in_s(E, 0);
    for (int e : net.open_edges) is_open[e] = 1;
    for (int e : sliced) in_s[e] = 1;
    while (true) {
        const int k = (int)sliced.size();
        const bool over = slice_cost_tl(tl, t, in_s).max_log2 > target;
        if (!over && k >= n_force) break;
        if (k >= 62) break;
        const int best = greedy_slice_step(net, t, tl, in_s, is_open, k, over);
        if (best < 0) break;
        in_s[best] = 1;
        sliced.push_back(best);
    }
    return sliced;
}

// Dynamic slicing (appendix A, "Dynamic slicing"): edges are sliced one at a
// time, each the greedy choice on the current tree, and after every sliced
// edge the tree is fine-tuned by subtree reconfiguration with the sliced legs
// removed (a few passes; a full re-tune at the end).  Stops when the largest
// intermediate meets the target and at least n_force edges are sliced.
std::vector<int> dynamic_slice(const Network& net, const std::vector<Legs>& leaf_legs, Tree& t, int target,
                               int n_force) {
    const int E = (int)net.edge_name.size();
    std::vector<int> sliced;
    std::vector<char> in_s(E, 0), is_open(E, 0);
    for (int e : net.open_edges) is_open[e] = 1;
    TreeLegs tl = tree_legs(net, t);
    while (true) {
        const int k = (int)sliced.size();
        const bool over = slice_cost_tl(tl, t, in_s).max_log2 > target;
        if ((!over && k >= n_force) || k >= 62) break;
        const int best = greedy_slice_step(net, t, tl, in_s, is_open, k, over);
        if (best < 0) break;
        in_s[best] = 1;
        sliced.push_back(best);
        t = reconfigure(leaf_legs, t, in_s, target, 8, 2);
        tl = tree_legs(net, t);
    }
    t = reconfigure(leaf_legs, t, in_s, target, 8, 16);
    return sliced;
}

struct BatchShape {
    double cmacs = 0, bytes = 0;
    int max_log2 = 0;
};

// Per-launch-sequence cost when the sliced edges in `in_b` are kept as batch
// legs (contracted together) and the rest of `in_s` are fixed.
BatchShape batch_shape(const TreeLegs& tl, const Tree& t, const std::vector<char>& in_s,
                       const std::vector<char>& in_b, int esize) {
    BatchShape bs;
    const int N = t.n_nodes();
    std::vector<Legs> lb(N);
    std::vector<char> dep(N, 0);
    for (int i = 0; i < t.n_leaves; ++i) {
        for (int e : tl.node[i]) {
            dep[i] |= in_s[e];
            if (!in_s[e] || in_b[e]) lb[i].push_back(e);
        }
    }
    for (size_t s = 0; s < t.lhs.size(); ++s) {
        int a = t.lhs[s], b = t.rhs[s], c = t.n_leaves + (int)s;
        dep[c] = dep[a] | dep[b];
        Legs both = set_inter(lb[a], lb[b]);
        Legs keep;
        for (int e : both)
            if (in_b[e]) keep.push_back(e);
        lb[c] = set_union(set_xor(lb[a], lb[b]), keep);
        if (!dep[c]) continue;
        int nb = (int)keep.size();
        int nk = (int)both.size() - nb;
        int nm = (int)lb[a].size() - (int)both.size();
        int nn = (int)lb[b].size() - (int)both.size();
        bs.cmacs += std::exp2((double)(nm + nn + nk + nb));
        bs.bytes += esize * (std::exp2((double)(nm + nk + nb)) + std::exp2((double)(nn + nk + nb)) +
                             std::exp2((double)(nm + nn + nb)));
        bs.max_log2 = std::max(bs.max_log2, (int)lb[c].size());
    }
    return bs;
}

int storage_bytes(tn_precision p) {
    switch (p) {
        case TN_C128: return 16;
        default: return 8;   // complex64 storage (also for the FP16/BF16 MFMA modes)
    }
}

}  // namespace

SliceCost slice_cost(const Network& net, const Tree& t, const std::vector<char>& in_s) {
    return slice_cost_tl(tree_legs(net, t), t, in_s);
}

// ------------------------------------------------------ layouts and steps

namespace {

// First-fit allocator over a linear arena (element units).
struct Arena {
    std::map<uint64_t, uint64_t> free_;   // offset -> length
    uint64_t top = 0, peak = 0;
    static uint64_t round(uint64_t n) { return (n + 63) & ~uint64_t(63); }
    uint64_t alloc(uint64_t n) {
        n = round(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                uint64_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > n) free_[off + n] = len - n;
                return off;
            }
        }
        uint64_t off = top;
        top += n;
        peak = std::max(peak, top);
        return off;
    }
    void release(uint64_t off, uint64_t n) {
        n = round(n);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
                it = pv;
            }
        }
        if (it->first + it->second == top) {
            top = it->first;
            free_.erase(it);
        }
    }
};

}  // namespace


// Batch legs: keep some sliced edges as legs so that 2^b slices are contracted
// in one launch sequence.  Planner-chosen slicings put the batch edges on the
// low slice bits; a caller's slicing keeps its order and batches a prefix.
static void choose_batch(const Network& net, const Tree& tree, const TreeLegs& tl, const tn_plan_opts& opts,
                         int esize, bool fixed_slicing, std::vector<int>& sliced, std::vector<int>& batch) {
    const int E = (int)net.edge_name.size();
    std::vector<char> in_s(E, 0), in_b(E, 0);
    for (int e : sliced) in_s[e] = 1;
    const int k = (int)sliced.size();
    const uint64_t cap = opts.max_workspace_bytes > 0 ? (uint64_t)opts.max_workspace_bytes : (uint64_t(32) << 30);
    const int want = opts.batch_log2;
    SliceCost sc = slice_cost_tl(tl, tree, in_s);
    const int size_cap = std::max(sc.max_log2, 30);   // 2^30 complex64 = 8 GiB per tensor of a launch group
    batch.clear();
    if (!fixed_slicing) {
        std::vector<int> chosen;
        while ((int)chosen.size() < k) {
            if (want >= 0 && (int)chosen.size() >= want) break;
            int best = -1;
            BatchShape bb;
            for (int e : sliced) {
                if (in_b[e]) continue;
                in_b[e] = 1;
                BatchShape x = batch_shape(tl, tree, in_s, in_b, esize);
                in_b[e] = 0;
                if (best < 0 || x.cmacs < bb.cmacs) {
                    best = e;
                    bb = x;
                }
            }
            if (best < 0) break;
            if (want < 0) {
                const double ws_est = 3.0 * std::exp2((double)bb.max_log2) * esize;
                if (bb.max_log2 > size_cap || ws_est > (double)cap || (int)chosen.size() >= 14) break;
            }
            in_b[best] = 1;
            chosen.push_back(best);
        }
        std::vector<int> reorder = chosen;
        for (int e : sliced)
            if (!in_b[e]) reorder.push_back(e);
        sliced = reorder;
        batch = chosen;
        return;
    }
    for (int i = 0; i < k; ++i) {   // caller's order: the largest prefix within the limits
        if (want >= 0 && i >= want) break;
        in_b[sliced[i]] = 1;
        BatchShape x = batch_shape(tl, tree, in_s, in_b, esize);
        const double ws_est = 3.0 * std::exp2((double)x.max_log2) * esize;
        if (want < 0 && (x.max_log2 > size_cap || ws_est > (double)cap || i >= 14)) break;
        batch.push_back(sliced[i]);
    }
}

static std::string finalize(Plan& p) {
    const Network& net = p.net;
    const Tree& t = p.tree;
    const int E = (int)net.edge_name.size();
    const int N = t.n_nodes();
    std::vector<char> in_s(E, 0), in_b(E, 0);
    std::vector<int> slice_bit(E, -1);
    for (size_t i = 0; i < p.sliced.size(); ++i) {
        in_s[p.sliced[i]] = 1;
        slice_bit[p.sliced[i]] = (int)i;
    }
    for (int e : p.batch) in_b[e] = 1;
    p.nodes.assign(N, NodeInfo());
    // legs with batch legs kept
    for (int i = 0; i < t.n_leaves; ++i) {
        Legs l = net.leaves[i].legs;
        std::sort(l.begin(), l.end());
        for (int e : l) {
            p.nodes[i].dep |= (bool)in_s[e];
            if (!in_s[e] || in_b[e]) p.nodes[i].legs.push_back(e);
        }
        if (i < (int)p.force_dep.size() && p.force_dep[i]) p.nodes[i].dep = true;
        p.nodes[i].home = HOME_LEAF;
    }
    for (size_t s = 0; s < t.lhs.size(); ++s) {
        int a = t.lhs[s], b = t.rhs[s], c = t.n_leaves + (int)s;
        NodeInfo& C = p.nodes[c];
        C.dep = p.nodes[a].dep || p.nodes[b].dep;
        Legs both = set_inter(p.nodes[a].legs, p.nodes[b].legs);
        Legs keep;
        for (int e : both)
            if (in_b[e]) keep.push_back(e);
        C.legs = set_union(set_xor(p.nodes[a].legs, p.nodes[b].legs), keep);
        p.nodes[a].parent = p.nodes[b].parent = c;
        C.home = C.dep ? HOME_WS : HOME_PLAN;
    }
    // root layout: result legs (bit 0 = last open leg) then batch legs in slice-bit order
    const int root = t.root();
    {
        Legs res = net.open_edges;
        std::reverse(res.begin(), res.end());
        Legs got = p.nodes[root].legs;
        Legs want = res;
        for (int e : p.batch) want.push_back(e);
        Legs ws = want;
        std::sort(ws.begin(), ws.end());
        if (ws != got) return "internal error: root legs are not open legs + batch legs";
        p.nodes[root].layout = want;
        p.root_log2 = (int)res.size();
    }
    // top-down layouts and step shapes
    p.steps.clear();
    std::vector<Step> by_node(N);
    for (int s = (int)t.lhs.size() - 1; s >= 0; --s) {
        const int c = t.n_leaves + s;
        int a = t.lhs[s], b = t.rhs[s];
        const Legs& la0 = p.nodes[a].legs;
        const Legs& lb0 = p.nodes[b].legs;
        const std::vector<int>& lc = p.nodes[c].layout;
        std::map<int, int> posc;
        for (size_t i = 0; i < lc.size(); ++i) posc[lc[i]] = (int)i;
        bool swap_ab = false;
        if (lb0.size() > la0.size()) swap_ab = true;
        else if (lb0.size() == la0.size() && !lc.empty()) {
            swap_ab = std::binary_search(lb0.begin(), lb0.end(), lc[0]) &&
                      !std::binary_search(la0.begin(), la0.end(), lc[0]);
        }
        if (swap_ab) std::swap(a, b);
        const Legs& la = p.nodes[a].legs;
        const Legs& lb = p.nodes[b].legs;
        Legs both = set_inter(la, lb);
        Legs bat, kk;
        for (int e : both) (in_b[e] ? bat : kk).push_back(e);
        Legs M = set_minus(la, lb), Nn = set_minus(lb, la);
        // order by position in C, batch edges last: batch legs then sit on
        // high address bits of every tensor, so the tiles (one batch index
        // each) always cover the lowest bits of their operands and outputs
        auto by_c = [&](Legs v) {
            std::sort(v.begin(), v.end(), [&](int x, int y) {
                if (in_b[x] != in_b[y]) return in_b[x] < in_b[y];
                return posc.at(x) < posc.at(y);
            });
            return v;
        };
        M = by_c(M);
        Nn = by_c(Nn);
        bat = by_c(bat);
        Step st{};
        st.node = c;
        st.a_node = a;
        st.b_node = b;
        st.m_log = (int)M.size();
        st.n_log = (int)Nn.size();
        st.k_log = (int)kk.size();
        st.b_log = (int)bat.size();
        for (int e : M) st.c_pos_m.push_back(posc.at(e));
        for (int e : Nn) st.c_pos_n.push_back(posc.at(e));
        for (int e : bat) st.c_pos_b.push_back(posc.at(e));
        st.invariant = !p.nodes[c].dep;
        std::vector<int> lay_a = M, lay_b = Nn;
        lay_a.insert(lay_a.end(), bat.begin(), bat.end());
        lay_a.insert(lay_a.end(), kk.begin(), kk.end());
        lay_b.insert(lay_b.end(), bat.begin(), bat.end());
        lay_b.insert(lay_b.end(), kk.begin(), kk.end());
        p.nodes[a].layout = lay_a;
        p.nodes[b].layout = lay_b;
        const double mnkb = (double)(st.m_log + st.n_log + st.k_log + st.b_log);
        st.cmacs = std::exp2(mnkb);
        st.bytes = p.esize * (std::exp2((double)(st.m_log + st.k_log + st.b_log)) +
                              std::exp2((double)(st.n_log + st.k_log + st.b_log)) +
                              std::exp2((double)(st.m_log + st.n_log + st.b_log)));
        choose_kernel(st.m_log, st.n_log, st.k_log, st.b_log, p.opts.prec, st.kernel, st.tile,
                      st.splitk_log);
        if (st.invariant && st.kernel == K_SPLITK) {   // computed once, outside any workspace
            st.kernel = K_SMALL;
            st.splitk_log = 0;
        }
        by_node[c] = st;
    }
    // leaves: outer-sliced legs on top
    for (int i = 0; i < t.n_leaves; ++i) {
        NodeInfo& L = p.nodes[i];
        if (t.n_nodes() == 1) L.layout = p.nodes[root].layout;
        std::vector<int> extra;
        for (int e : net.leaves[i].legs)
            if (in_s[e] && !in_b[e]) extra.push_back(e);
        std::sort(extra.begin(), extra.end(), [&](int x, int y) { return slice_bit[x] < slice_bit[y]; });
        for (int e : extra) {
            L.layout.push_back(e);
            L.sliced_bits.push_back(slice_bit[e]);
        }
    }
    // execution order: invariant steps first, then dependent steps
    for (int pass = 0; pass < 2; ++pass)
        for (size_t s = 0; s < t.lhs.size(); ++s) {
            const Step& st = by_node[t.n_leaves + s];
            if ((pass == 0) == st.invariant) p.steps.push_back(st);
        }
    p.n_invariant_steps = 0;
    for (auto& st : p.steps) p.n_invariant_steps += st.invariant;
    p.step_of_node.assign(N, -1);
    for (size_t i = 0; i < p.steps.size(); ++i) p.step_of_node[p.steps[i].node] = (int)i;
    // memory: plan arena holds leaves and invariant tensors; the workspace
    // holds dependent intermediates with liveness reuse plus split-K scratch
    uint64_t plan_top = 0;
    for (int i = 0; i < t.n_leaves; ++i) {
        p.nodes[i].off = plan_top;
        plan_top += Arena::round(uint64_t(1) << p.nodes[i].layout.size());
    }
    for (auto& st : p.steps)
        if (st.invariant) {
            p.nodes[st.node].off = plan_top;
            st.c_off = plan_top;
            plan_top += Arena::round(uint64_t(1) << p.nodes[st.node].legs.size());
        }
    p.plan_elems = plan_top;
    // max-magnitude slots: leaves, then invariant tensors, then dependent ones
    {
        int next = 0;
        for (int i = 0; i < t.n_leaves; ++i) p.nodes[i].slot = next++;
        for (auto& st : p.steps)
            if (st.invariant) p.nodes[st.node].slot = next++;
        p.n_static_slots = next;
        for (auto& st : p.steps)
            if (!st.invariant) p.nodes[st.node].slot = next++;
    }
    Arena ws;
    for (auto& st : p.steps) {
        if (st.invariant) continue;
        const uint64_t csz = uint64_t(1) << p.nodes[st.node].legs.size();
        st.c_off = ws.alloc(csz);
        p.nodes[st.node].off = st.c_off;
        if (st.kernel == K_SPLITK) {
            // partial tiles are stored at the storage width
            const uint64_t scr_elems = uint64_t(1) << (st.m_log + st.n_log + st.b_log + st.splitk_log);
            st.scratch_off = ws.alloc(scr_elems);
            ws.release(st.scratch_off, scr_elems);
        }
        bool panel_any = false;
        for (int t = 0; t < kNumPanelTiles; ++t)
            panel_any |= panel_ok(st.m_log, st.n_log, st.k_log, st.b_log, p.opts.prec, t);
        if (lp_prec(p.opts.prec) && panel_any) {
            // hi and lo word planes of A: 8 bytes per element, one storage element each
            const uint64_t conv = uint64_t(1) << (st.m_log + st.k_log + st.b_log);
            st.conv_off = ws.alloc(conv);
            ws.release(st.conv_off, conv);
        }
        for (int o : {st.a_node, st.b_node})
            if (p.nodes[o].home == HOME_WS) ws.release(p.nodes[o].off, uint64_t(1) << p.nodes[o].legs.size());
    }
    p.ws_elems = std::max<uint64_t>(ws.peak, 64);
    if (t.n_nodes() == 1) p.ws_elems = std::max<uint64_t>(p.ws_elems, uint64_t(1) << p.nodes[root].legs.size());
    return "";
}

static void fill_stats(Plan& p) {
    tn_plan_stats& s = p.stats;
    s = tn_plan_stats{};
    s.n_sliced = (int)p.sliced.size();
    s.n_slices = uint64_t(1) << s.n_sliced;
    s.batch_log2 = p.batch_log2;
    s.n_open = (int)p.net.open_edges.size();
    s.n_leaves = p.tree.n_leaves;
    s.n_steps = (int)p.tree.lhs.size();
    s.acc_log2 = p.root_log2;
    double per_batch = 0, inv = 0, bytes = 0;
    int mx = 0;
    for (auto& st : p.steps) {
        if (st.invariant) inv += st.cmacs;
        else {
            per_batch += st.cmacs;
            bytes += st.bytes;
        }
        if (st.kernel == K_MFMA || st.kernel == K_SKINNY || st.kernel == K_PANEL) s.n_dense_steps++;
        else s.n_small_steps++;   // streaming, VALU tile and split-K
    }
    for (int c = p.tree.n_leaves; c < p.tree.n_nodes(); ++c)
        mx = std::max(mx, (int)p.nodes[c].legs.size() - (p.nodes[c].dep ? 0 : 0));
    const double B = std::exp2((double)p.batch_log2);
    s.cmacs_per_batch = per_batch;
    s.bytes_per_batch = bytes + 16.0 * std::exp2((double)p.root_log2);
    s.cmacs_per_slice = per_batch / B;
    s.cmacs_per_slice_unmerged = p.unmerged_cmacs_per_slice;
    s.cmacs_invariant = inv;
    s.cmacs_tail = 0;
    s.bytes_per_slice = s.bytes_per_batch / B;
    s.max_log2_size = mx - p.batch_log2 > 0 ? mx : mx;
    // per-slice max: legs without batch legs
    int mx1 = 0;
    std::set<int> bset(p.batch.begin(), p.batch.end());
    for (int c = p.tree.n_leaves; c < p.tree.n_nodes(); ++c) {
        int n = 0;
        for (int e : p.nodes[c].legs) n += !bset.count(e);
        mx1 = std::max(mx1, n);
    }
    s.max_log2_size = mx1;
    s.workspace_bytes = p.ws_elems * (uint64_t)p.esize;
    s.tail_workspace_bytes = 0;
    s.n_c = 0;
}

// Planning pipeline on a built network (out.net, out.opts and out.esize set).
double dense_step_rate(tn_precision prec) {
    // dense steps measured on the 40-qubit workload: FP32 MFMA panels about
    // 110 TFLOP/s, the split-FP16 panel about 200 on compute-bound shapes.
    // BF16 (245 there) keeps the FP32 figure: its plan re-tuned with 245 ran
    // 7 % slower per launch group.  Complex128 keeps it too (not measured).
    return prec == TN_SPLIT_FP16 ? 200e12 : 110e12;
}

double write_weight(tn_precision prec) {
    // Writes stream at about half the rate of reads on MI355X (a plain device
    // copy moves 2.65 TB/s each way).  Counting output bytes twice in the time
    // objective made the split-FP16 plan of the 40-qubit workload 1.32x
    // faster per launch group (its steps are bound by memory, not by the
    // matrix cores) but the complex64 plan 3 % slower and the 25-qubit
    // complex64 job 22 % slower, so the low-precision forms use it and
    // complex64 / complex128 do not.
    return lp_prec(prec) ? 2.0 : 1.0;
}

// Roofline time estimate (seconds) of one job on a finalized plan: per
// launch max(8 cmacs / rate, bytes / 4 TB/s) + 2 us, slice-dependent steps
// once per launch group, invariant steps once.
static double plan_time_estimate(const Plan& p) {
    const double groups = std::exp2((double)p.sliced.size() - p.batch_log2);
    const double dense = dense_step_rate(p.opts.prec);
    double t = 0;
    for (const Step& st : p.steps) {
        const bool mfma = st.kernel == K_MFMA || st.kernel == K_PANEL || st.kernel == K_SKINNY;
        const double out_bytes = p.esize * std::exp2((double)(st.m_log + st.n_log + st.b_log));
        const double bytes = st.bytes + (write_weight(p.opts.prec) - 1.0) * out_bytes;
        const double one = std::max(8.0 * st.cmacs / (mfma ? dense : 25e12), bytes / 4e12) + 2e-6;
        t += st.invariant ? one : one * groups;
    }
    return t;
}

static std::string plan_network(Plan& out, const tn_tree* tree, const std::vector<int>& user_sliced,
                                bool fixed_slicing, const CostModel* cm, const Tree* extra = nullptr) {
    const tn_plan_opts& opts = out.opts;
    const Network& net = out.net;
    const int E = (int)net.edge_name.size();
    const int L = (int)net.leaves.size();
    std::string err;
    std::vector<Legs> leaf_legs(L);
    for (int i = 0; i < L; ++i) {
        leaf_legs[i] = net.leaves[i].legs;
        std::sort(leaf_legs[i].begin(), leaf_legs[i].end());
    }
    // candidate trees
    std::vector<Tree> cands;
    if (tree) {
        if (tree->n_steps != L - 1) return "tree must have n_leaves - 1 steps";
        Tree t;
        t.n_leaves = L;
        std::vector<char> used(2 * L, 0);
        for (int s = 0; s < tree->n_steps; ++s) {
            int a = tree->lhs[s], b = tree->rhs[s];
            if (a < 0 || b < 0 || a >= L + s || b >= L + s || a == b || used[a] || used[b])
                return "invalid tree at step " + std::to_string(s);
            used[a] = used[b] = 1;
            t.lhs.push_back(a);
            t.rhs.push_back(b);
        }
        cands.push_back(t);
    } else {
        // candidates alternate between hierarchical bipartition (appendix A)
        // and randomised greedy orders; the cheapest after slicing is kept
        const int R = std::max(1, opts.restarts);
        std::mt19937_64 rng(opts.seed + 777);
        std::uniform_real_distribution<double> ua(0.5, 1.5), ut(0.0, 1.0), ue(0.05, 0.7);
        std::uniform_int_distribution<int> ul(3, 16);
        cands.push_back(time_order_tree(L));
        for (int r = 0; r < R; ++r) {
            if (r % 4 == 2) {
                const double eps = r == 0 ? 0.3 : ue(rng);
                const int leaf = r == 0 ? 8 : ul(rng);
                const int open_w = r == 0 ? 2 : (int)(rng() % 4);
                cands.push_back(partition_tree(leaf_legs, opts.seed * 1000003ULL + r, eps, leaf, open_w));
            } else {
                double alpha = r == 1 ? 1.0 : ua(rng);
                double temp = r == 1 ? 0.0 : ut(rng);
                cands.push_back(greedy_tree(leaf_legs, opts.seed * 1000003ULL + r, alpha, temp));
            }
        }
        // hierarchical bipartition under time and space caps on every
        // bisection (appendix A): the space cap is the memory target plus a
        // slicing budget of 4, 8 or 12 legs, the time cap 8 above it
        for (int r = 0; r < (R + 3) / 4; ++r) {
            const int space_cap = opts.max_log2_size + 4 * (1 + r % 3);
            const double eps = r == 0 ? 0.3 : ue(rng);
            const int leaf = r == 0 ? 60 : ul(rng);   // the paper's finest sub-graphs hold up to 60 tensors
            const int open_w = r == 0 ? 2 : (int)(rng() % 4);
            cands.push_back(partition_tree(leaf_legs, opts.seed * 1000003ULL + 7919 + r, eps, leaf, open_w,
                                           space_cap + 8, space_cap));
        }
        if (extra && extra->n_leaves == L) cands.push_back(*extra);
    }
    if (L == 1) {
        cands.clear();
        Tree t;
        t.n_leaves = 1;
        cands.push_back(t);
    }
    // slice each candidate; rank by FLOP count (or by the learned model)
    double best_cost = -1;
    const int n_force = fixed_slicing ? 0 : std::max(0, opts.n_slice_edges);
    struct Ranked {
        Tree t;
        std::vector<int> s;
        double flops, unmerged;
    };
    std::vector<Ranked> ranked;
    for (auto& t : cands) {
        std::vector<char> in_s(E, 0);
        if (!tree) {   // local optimisation of the unsliced tree
            if (fixed_slicing)
                for (int e : user_sliced) in_s[e] = 1;
            t = reconfigure(leaf_legs, t, in_s, fixed_slicing ? opts.max_log2_size : 64, 8, 16);
        }
        // dynamic slicing (re-tune after every sliced edge) on a copy of the
        // tree; compared below with one-shot slicing plus one re-tune
        Tree t_dyn = t;
        std::vector<int> s_dyn;
        const bool try_dyn = !tree && !fixed_slicing && opts.slicing != 1;
        const bool try_one = tree || fixed_slicing || opts.slicing != 2;
        if (try_dyn) s_dyn = dynamic_slice(net, leaf_legs, t_dyn, opts.max_log2_size, n_force);
        TreeLegs tl = tree_legs(net, t);
        std::vector<int> s = fixed_slicing ? user_sliced
                                           : (try_one ? greedy_slice(net, t, tl, opts.max_log2_size, n_force, {})
                                                      : std::vector<int>());
        for (int e : s) in_s[e] = 1;
        if (!tree && !fixed_slicing && try_one && !s.empty()) {
            // re-tune the tree for one slice, then top up the slicing if needed
            Tree t2 = reconfigure(leaf_legs, t, in_s, opts.max_log2_size, 8, 16);
            TreeLegs tl2 = tree_legs(net, t2);
            std::vector<int> s2 = greedy_slice(net, t2, tl2, opts.max_log2_size, n_force, s);
            std::vector<char> in2(E, 0);
            for (int e : s2) in2[e] = 1;
            if (slice_cost_tl(tl2, t2, in2).total((int)s2.size()) <
                slice_cost_tl(tl, t, in_s).total((int)s.size())) {
                t = t2;
                tl = tl2;
                s = s2;
                in_s = in2;
            }
        }
        if (try_dyn) {
            TreeLegs tld = tree_legs(net, t_dyn);
            std::vector<char> ind(E, 0);
            for (int e : s_dyn) ind[e] = 1;
            const SliceCost scd = slice_cost_tl(tld, t_dyn, ind);
            if (!try_one || (scd.max_log2 <= opts.max_log2_size &&
                             scd.total((int)s_dyn.size()) < slice_cost_tl(tl, t, in_s).total((int)s.size()))) {
                t = t_dyn;
                tl = tld;
                s = s_dyn;
                in_s = ind;
            }
        }
        SliceCost sc = slice_cost_tl(tl, t, in_s);
        double cost = sc.total((int)s.size());
        if (std::getenv("TN_DEBUG_CANDS")) {
            std::vector<char> none(E, 0);
            SliceCost raw = slice_cost_tl(tl, t, none);
            std::fprintf(stderr, "cand %zu: raw max %d log2 %.2f | k %zu log2 total %.2f\n",
                         (size_t)(&t - &cands[0]), raw.max_log2, std::log2(raw.invariant), s.size(), std::log2(cost));
        }
        ranked.push_back({t, s, cost, sc.per_slice});
        if (best_cost < 0 || cost < best_cost) {
            best_cost = cost;
            out.tree = t;
            out.sliced = s;
            out.unmerged_cmacs_per_slice = sc.per_slice;
        }
    }
    out.stats.n_candidates = (int)ranked.size();
    int model_used = 0;
    double predicted = 0;
    bool mlp_chose = false;
    if (opts.cost_model == 1 && cm && cm->predict) {
        // Learned model: predicted time of the whole job for plan variants
        // that differ in ways the multiply-add count does not see: the four
        // cheapest candidates by FLOP count, each as sliced and, with branch
        // merging on, re-tuned for estimated time (merged).  Every variant is
        // finalized (batch legs, layouts, kernel per step) and each executed
        // step is one row of features; variants with a row outside the
        // model's training support are left out.
        std::vector<size_t> idx(ranked.size());
        for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
        std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return ranked[a].flops < ranked[b].flops; });
        struct Var {
            Tree t;
            std::vector<int> s;
            double unmerged;
            Plan p;
        };
        std::vector<Var> vars;
        const double rate = dense_step_rate(opts.prec);
        for (size_t i = 0; i < std::min<size_t>(4, idx.size()); ++i) {
            const Ranked& r = ranked[idx[i]];
            vars.push_back({r.t, r.s, r.unmerged, Plan()});
            if (opts.branch_merge && !tree) {
                std::vector<char> in_s(E, 0);
                for (int e : r.s) in_s[e] = 1;
                Tree m = reconfigure(leaf_legs, r.t, in_s, opts.max_log2_size, 8, 16, 1, out.esize, rate,
                                     write_weight(opts.prec));
                TreeLegs tlm = tree_legs(net, m);
                if (slice_cost_tl(tlm, m, in_s).max_log2 <= opts.max_log2_size &&
                    (m.lhs != r.t.lhs || m.rhs != r.t.rhs))
                    vars.push_back({m, r.s, r.unmerged, Plan()});
            }
        }
        std::vector<float> feats;
        std::vector<std::pair<size_t, size_t>> span;
        std::vector<char> usable(vars.size(), 0);
        for (size_t v = 0; v < vars.size(); ++v) {
            Plan& pv = vars[v].p;
            pv = out;
            pv.tree = vars[v].t;
            pv.sliced = vars[v].s;
            TreeLegs tlv = tree_legs(net, pv.tree);
            choose_batch(net, pv.tree, tlv, opts, out.esize, fixed_slicing, pv.sliced, pv.batch);
            pv.batch_log2 = (int)pv.batch.size();
            const size_t r0 = feats.size() / kStepFeatures;
            span.push_back({r0, 0});
            if (!finalize(pv).empty()) continue;
            bool inside = true;
            for (const Step& st : pv.steps) {
                float f[kStepFeatures];
                step_features(st.m_log, st.n_log, st.k_log, st.b_log, st.kernel, out.esize, f);
                if (cm->in_support && !cm->in_support(f)) inside = false;
                feats.insert(feats.end(), f, f + kStepFeatures);
            }
            span.back().second = pv.steps.size();
            if (!inside) {
                feats.resize(r0 * kStepFeatures);
                span.back().second = 0;
                continue;
            }
            usable[v] = 1;
        }
        size_t n_usable = 0;
        for (char u : usable) n_usable += u;
        if (n_usable == 0) {
            model_used = 2;
        } else {
            std::vector<float> pred;
            std::string e = cm->predict(feats, (int)(feats.size() / kStepFeatures), pred);
            if (!e.empty()) return "cost model: " + e;
            double best = -1;
            size_t bi = 0;
            for (size_t v = 0; v < vars.size(); ++v) {
                if (!usable[v]) continue;
                const Plan& pv = vars[v].p;
                double dep_ms = 0, inv_ms = 0;
                for (size_t i = 0; i < span[v].second; ++i) {
                    const double ms = std::exp((double)pred[span[v].first + i]);
                    (pv.steps[i].invariant ? inv_ms : dep_ms) += ms;
                }
                const double tot = std::exp2((double)pv.sliced.size() - pv.batch_log2) * dep_ms + inv_ms;
                if (std::getenv("TN_DEBUG_CANDS"))
                    std::fprintf(stderr, "mlp variant %zu: predicted %.3f ms per job\n", v, tot);
                if (best < 0 || tot < best) {
                    best = tot;
                    bi = v;
                }
            }
            out.tree = vars[bi].t;
            out.sliced = vars[bi].s;
            out.unmerged_cmacs_per_slice = vars[bi].unmerged;
            predicted = best;
            model_used = 1;
            mlp_chose = true;
            out.stats.n_candidates = (int)n_usable;
        }
    }
    {
        TreeLegs tl = tree_legs(net, out.tree);
        choose_batch(net, out.tree, tl, opts, out.esize, fixed_slicing, out.sliced, out.batch);
        out.batch_log2 = (int)out.batch.size();
    }
    if (out.sliced.size() > 62) return "more than 62 sliced edges needed";
    // branch merging: re-tune the chosen tree for estimated time per slice
    // (more multiply-adds, fewer skinny steps); kept only if faster
    if (opts.branch_merge && !tree && !mlp_chose) {
        std::vector<char> in_s(E, 0);
        for (int e : out.sliced) in_s[e] = 1;
        const double rate = dense_step_rate(opts.prec);
        const double ww = write_weight(opts.prec);
        Tree merged = reconfigure(leaf_legs, out.tree, in_s, opts.max_log2_size, 8, 16, 1, out.esize, rate, ww);
        TreeLegs tlm = tree_legs(net, merged);
        if (slice_cost_tl(tlm, merged, in_s).max_log2 <= opts.max_log2_size &&
            tree_time_estimate(leaf_legs, merged, in_s, out.esize, rate, ww) <
                tree_time_estimate(leaf_legs, out.tree, in_s, out.esize, rate, ww)) {
            // the per-slice estimate ignores batch legs (work shared by the
            // slices of a launch group, outputs that keep the batch legs) and
            // the slice-invariant part: confirm on the executed steps of both
            // trees, one whole job each
            Plan a = out, b = out;
            b.tree = merged;
            std::string ea = finalize(a), eb = finalize(b);
            if (!ea.empty()) return ea;
            if (std::getenv("TN_DEBUG_CANDS"))
                std::fprintf(stderr, "merge: unmerged %.3f ms, merged %.3f ms (estimated)\n",
                             1e3 * plan_time_estimate(a), eb.empty() ? 1e3 * plan_time_estimate(b) : -1.0);
            if (eb.empty() && plan_time_estimate(b) < plan_time_estimate(a)) out.tree = merged;
        }
    }
    err = finalize(out);
    if (!err.empty()) return err;
    const int n_cand = out.stats.n_candidates;
    fill_stats(out);
    out.stats.n_candidates = n_cand;
    out.stats.cost_model_used = model_used;
    out.stats.predicted_ms = predicted;
    return "";
}

// Big-head split (section "Big-head simulation of quantum circuits", Fig. 1):
// the tail is a set of leaves holding every open leg, grown greedily from the
// leaves with open legs (adjacent leaf of smallest cut change, plateaus
// allowed, at most half the network; the smallest cut seen is kept);
// n_c is bounded so that the head's accumulator stays within 2^28 entries.
static std::vector<char> choose_tail(const Network& net, int max_log2) {
    const int L = (int)net.leaves.size();
    const int E = (int)net.edge_name.size();
    std::vector<char> is_open(E, 0), in_t(L, 0);
    for (int e : net.open_edges) is_open[e] = 1;
    std::vector<std::vector<int>> ends(E);
    for (int i = 0; i < L; ++i)
        for (int e : net.leaves[i].legs) ends[e].push_back(i);
    for (int i = 0; i < L; ++i)
        for (int e : net.leaves[i].legs)
            if (is_open[e]) in_t[i] = 1;
    // change of the cut when leaf i joins the tail: its legs to tail leaves
    // leave the cut, its legs to head leaves enter it
    auto delta = [&](int i) {
        int d = 0;
        for (int e : net.leaves[i].legs) {
            if (ends[e].size() != 2) continue;
            const int j = ends[e][0] == i ? ends[e][1] : ends[e][0];
            d += in_t[j] ? -1 : 1;
        }
        return d;
    };
    int cut = 0, n_t = 0;
    for (int e = 0; e < E; ++e)
        if (ends[e].size() == 2 && in_t[ends[e][0]] != in_t[ends[e][1]]) ++cut;
    for (int i = 0; i < L; ++i) n_t += in_t[i];
    const int n_open = (int)net.open_edges.size();
    // grow by the adjacent leaf of smallest cut change (ties: lowest id),
    // plateaus included, up to half the network; keep the smallest cut seen
    std::vector<char> best_t = in_t;
    int best_cut = cut;
    while (2 * (n_t + 1) <= L) {
        int pick = -1, pick_d = 0;
        for (int i = 0; i < L; ++i) {
            if (in_t[i]) continue;
            bool adj = false;
            for (int e : net.leaves[i].legs)
                for (int j : ends[e]) adj |= (j != i && in_t[j]);
            if (!adj) continue;
            const int d = delta(i);
            if (pick < 0 || d < pick_d) {
                pick = i;
                pick_d = d;
            }
        }
        if (pick < 0 || pick_d > 0) break;
        in_t[pick] = 1;
        ++n_t;
        cut += pick_d;
        if (cut < best_cut) {
            best_cut = cut;
            best_t = in_t;
        }
    }
    (void)n_open;
    if (best_cut > max_log2) return {};
    return best_t;
}

// A network over a subset of leaves with the given open edges (edge ids and
// names are those of the full network).
static Network sub_network(const Network& net, const std::vector<char>& keep, const std::vector<int>& open) {
    Network s;
    s.n_qubits = net.n_qubits;
    s.edge_name = net.edge_name;
    s.end0.assign(net.edge_name.size(), -1);
    s.end1.assign(net.edge_name.size(), -1);
    for (size_t i = 0; i < net.leaves.size(); ++i)
        if (keep[i]) {
            const int id = (int)s.leaves.size();
            s.leaves.push_back(net.leaves[i]);
            for (int e : net.leaves[i].legs) {
                if (s.end0[e] < 0) s.end0[e] = id;
                else s.end1[e] = id;
            }
        }
    s.open_edges = open;
    return s;
}

std::string make_plan(const tn_circuit& c, const std::vector<int>& open_q,
                      const std::vector<int>& fixed_q, const std::vector<uint8_t>& bits,
                      const tn_tree* tree, const tn_edge* sliced, int n_sliced,
                      const tn_plan_opts& opts, Plan& out, const CostModel* cm) {
    out = Plan();
    out.opts = opts;
    if (opts.prec < TN_C64 || opts.prec > TN_BF16) return "unknown precision";
    if (opts.max_log2_size < 1 || opts.max_log2_size > 40) return "max_log2_size out of range";
    out.esize = storage_bytes(opts.prec);
    Network full;
    std::string err = build_network(c, open_q, fixed_q, bits, full);
    if (!err.empty()) return err;
    const int E = (int)full.edge_name.size();
    std::vector<int> user_sliced;
    if (sliced && n_sliced > 0) {
        std::vector<char> seen(E, 0), is_open(E, 0);
        for (int e : full.open_edges) is_open[e] = 1;
        for (int i = 0; i < n_sliced; ++i) {
            int e = full.find_edge(sliced[i].qubit, sliced[i].segment);
            if (e < 0) return "sliced edge (" + std::to_string(sliced[i].qubit) + "," +
                              std::to_string(sliced[i].segment) + ") is not an edge";
            if (is_open[e]) return "an open leg cannot be sliced";
            if (seen[e]) return "sliced edge repeated";
            seen[e] = 1;
            user_sliced.push_back(e);
        }
    }
    if (!opts.bighead) {
        out.net = std::move(full);
        return plan_network(out, tree, user_sliced, n_sliced >= 0, cm);
    }
    // big-head: head over the leaves outside the tail, whose result
    // v_head[c] (c = the cut legs) is summed over all slices; at the end the
    // tail network plus one leaf holding v_head is contracted once, in
    // complex128, straight into A[s2] = sum_c T_tail[s2, c] v_head[c]
    if (tree || (sliced && n_sliced > 0)) return "bighead: the planner chooses the tree and the sliced edges";
    // Tail candidates: (1) the leaves under the lowest node of the best
    // full-network order that holds every open leg (the order is found
    // first and the bottleneck read off it), when that node is not the
    // root; (2) the greedy smallest-cut tail.  The cheaper split (head over
    // all slices plus tail once) is kept.
    Plan fullp;
    fullp.opts = opts;
    fullp.opts.bighead = 0;
    fullp.esize = out.esize;
    fullp.net = full;
    err = plan_network(fullp, nullptr, {}, false, cm);
    if (!err.empty()) return err;
    std::vector<std::pair<std::vector<char>, Tree>> tails;   // tail leaves, induced head order
    {
        const Tree& ft = fullp.tree;
        const int L = ft.n_leaves, N = ft.n_nodes();
        std::vector<char> has_open(L, 0);
        {
            std::vector<char> is_open(E, 0);
            for (int e : full.open_edges) is_open[e] = 1;
            for (int i = 0; i < L; ++i)
                for (int e : full.leaves[i].legs) has_open[i] |= is_open[e];
        }
        int total = 0;
        for (int i = 0; i < L; ++i) total += has_open[i];
        std::vector<int> cnt(N, 0);
        for (int i = 0; i < L; ++i) cnt[i] = has_open[i];
        for (int k = 0; k < (int)ft.lhs.size(); ++k) cnt[L + k] = cnt[ft.lhs[k]] + cnt[ft.rhs[k]];
        int lca = -1;
        for (int v = 0; v < N && total > 0; ++v)
            if (cnt[v] == total) {
                lca = v;
                break;
            }
        if (lca >= 0 && lca != ft.root()) {
            std::vector<char> under(N, 0), in_t(L, 0);
            under[lca] = 1;
            for (int k = (int)ft.lhs.size() - 1; k >= 0; --k)
                if (under[L + k]) under[ft.lhs[k]] = under[ft.rhs[k]] = 1;
            for (int i = 0; i < L; ++i) in_t[i] = under[i];
            tails.push_back({in_t, Tree()});
        }
    }
    {
        std::vector<char> g = choose_tail(full, 28);
        if (!g.empty()) tails.push_back({g, Tree()});
    }
    // each head also gets the full order restricted to its leaves as a candidate
    for (auto& cand : tails) {
        const Tree& ft = fullp.tree;
        const int L = ft.n_leaves, N = ft.n_nodes();
        std::vector<int> map(N, -1);
        Tree& ht = cand.second;
        ht = Tree();
        for (int i = 0; i < L; ++i)
            if (!cand.first[i]) map[i] = ht.n_leaves++;
        for (int k = 0; k < (int)ft.lhs.size(); ++k) {
            const int a = map[ft.lhs[k]], b = map[ft.rhs[k]];
            if (a >= 0 && b >= 0) {
                map[L + k] = ht.n_leaves + (int)ht.lhs.size();
                ht.lhs.push_back(a);
                ht.rhs.push_back(b);
            } else {
                map[L + k] = a >= 0 ? a : b;
            }
        }
    }
    if (tails.empty()) return "bighead: no tail with at most 28 cut legs found";
    std::string last_err = "bighead: no tail with at most 28 cut legs found";
    double best = -1;
    for (auto& cand : tails) {
        const std::vector<char>& in_t = cand.first;
        std::vector<char> in_h(in_t.size());
        for (size_t i = 0; i < in_t.size(); ++i) in_h[i] = !in_t[i];
        std::vector<int> cut;
        {
            std::vector<int> cnt_t(E, 0), cnt_h(E, 0);
            for (size_t i = 0; i < full.leaves.size(); ++i)
                for (int e : full.leaves[i].legs) (in_t[i] ? cnt_t : cnt_h)[e]++;
            for (int e = 0; e < E; ++e)
                if (cnt_t[e] == 1 && cnt_h[e] == 1) cut.push_back(e);
        }
        const int n_c = (int)cut.size();
        if (n_c > 28) continue;
        Plan h;
        h.opts = opts;
        h.esize = out.esize;
        h.net = sub_network(full, in_h, cut);   // accumulator index: cut[0] most significant
        Network tail_net = sub_network(full, in_t, full.open_edges);
        {
            HostTensor v;   // address bit j <-> cut[n_c - 1 - j], as in the head's accumulator
            for (int j = n_c - 1; j >= 0; --j) v.legs.push_back(cut[j]);
            v.data.assign(size_t(1) << n_c, cd(0.0, 0.0));
            tail_net.leaves.push_back(std::move(v));
        }
        h.full_open = full.open_edges;
        err = plan_network(h, nullptr, {}, false, cm, cand.second.n_leaves ? &cand.second : nullptr);
        if (!err.empty()) {
            last_err = "head: " + err;
            continue;
        }
        h.tail = std::make_shared<Plan>();
        Plan& t = *h.tail;
        t.opts = opts;
        t.opts.prec = TN_C128;       // contracted once per tn_amplitudes call: full precision
        t.opts.bighead = 0;
        t.opts.batch_log2 = 0;
        t.opts.branch_merge = 0;
        t.opts.max_log2_size = 40;
        t.esize = storage_bytes(TN_C128);
        t.net = std::move(tail_net);
        t.force_dep.assign(t.net.leaves.size(), 0);
        t.force_dep.back() = 1;
        err = plan_network(t, nullptr, {}, true, nullptr);
        if (!err.empty()) {
            last_err = "tail: " + err;
            continue;
        }
        h.stats.n_c = n_c;
        h.stats.n_open = (int)h.full_open.size();
        h.stats.cmacs_tail = t.stats.cmacs_invariant + t.stats.cmacs_per_slice;
        h.stats.tail_workspace_bytes = std::max<uint64_t>(t.stats.workspace_bytes, 256);
        const double cost = h.stats.cmacs_invariant + double(h.stats.n_slices) * h.stats.cmacs_per_slice +
                            h.stats.cmacs_tail;
        if (std::getenv("TN_DEBUG_CANDS"))
            std::fprintf(stderr, "bighead tail %zu: n_c %d cost %.3e\n", (size_t)(&cand - &tails[0]), n_c, cost);
        if (best < 0 || cost < best) {
            best = cost;
            out = std::move(h);
        }
    }
    if (best < 0) return last_err;
    return "";
}

// Open qubits read off a contraction order (section "Big-head simulation of
// quantum circuits": the order is found first, then the open qubits are
// chosen from it).  The network with every qubit closed is ordered like any
// other; each qubit ends at its last two-qubit gate (or at its own node if it
// has none).  Among the tree nodes with at most half of the leaves under them
// whose subtree holds the ends of at least n_open qubits, the one with the
// fewest legs to the rest of the network (ties: fewest leaves) is the tail; n_open of its qubits (lowest ids) are opened, and its
// leg count is the head-tail cut.
std::string choose_open_qubits(const tn_circuit& c, int n_open, const tn_plan_opts& opts, std::vector<int>& open_out,
                               int& cut_out) {
    const int n = c.n_qubits;
    if (n <= 0 || n > 4096) return "n_qubits out of range";
    if (n_open < 1 || n_open > std::min(n, 40)) return "n_open out of range";
    Plan p;
    p.opts = opts;
    p.opts.bighead = 0;
    if (p.opts.prec < TN_C64 || p.opts.prec > TN_BF16) return "unknown precision";
    if (p.opts.max_log2_size < 1 || p.opts.max_log2_size > 40) return "max_log2_size out of range";
    p.esize = storage_bytes(p.opts.prec);
    std::vector<int> all(n);
    for (int q = 0; q < n; ++q) all[q] = q;
    std::string err = build_network(c, {}, all, std::vector<uint8_t>(n, 0), p.net);
    if (!err.empty()) return err;
    std::vector<int> end_leaf(n, -1);
    int n2 = 0;
    for (int g = 0; g < c.n_gates; ++g)
        if (c.gates[g].q1 >= 0) {
            end_leaf[c.gates[g].q0] = end_leaf[c.gates[g].q1] = n2;
            ++n2;
        }
    int extra = 0;
    for (int q = 0; q < n; ++q)
        if (end_leaf[q] < 0) end_leaf[q] = n2 + extra++;
    if ((int)p.net.leaves.size() != n2 + extra) return "internal error: leaf count";
    err = plan_network(p, nullptr, {}, false, nullptr);
    if (!err.empty()) return err;
    const Tree& t = p.tree;
    const int L = t.n_leaves, N = t.n_nodes();
    const TreeLegs tl = tree_legs(p.net, t);
    std::vector<int> ends(N, 0), leaves(N, 0);
    for (int q = 0; q < n; ++q) ends[end_leaf[q]]++;
    for (int i = 0; i < L; ++i) leaves[i] = 1;
    for (int k = 0; k < (int)t.lhs.size(); ++k) {
        ends[L + k] = ends[t.lhs[k]] + ends[t.rhs[k]];
        leaves[L + k] = leaves[t.lhs[k]] + leaves[t.rhs[k]];
    }
    int best = -1;
    for (int v = 0; v < N; ++v) {
        // the tail is the small side: at most half of the leaves
        if (ends[v] < n_open || 2 * leaves[v] > L) continue;
        if (N == 1) break;
        const size_t cut = tl.node[v].size();
        if (best < 0 || cut < tl.node[best].size() || (cut == tl.node[best].size() && leaves[v] < leaves[best]))
            best = v;
    }
    if (best < 0) best = t.root();   // no subtree of at most half the leaves holds enough ends
    std::vector<char> under(N, 0);
    under[best] = 1;
    for (int k = (int)t.lhs.size() - 1; k >= 0; --k)
        if (under[L + k]) under[t.lhs[k]] = under[t.rhs[k]] = 1;
    open_out.clear();
    for (int q = 0; q < n && (int)open_out.size() < n_open; ++q)
        if (under[end_leaf[q]]) open_out.push_back(q);
    cut_out = (int)tl.node[best].size();
    return "";
}

// ------------------------------------------------------------------- JSON

std::string plan_to_json(const Plan& p) {
    std::ostringstream o;
    auto edge = [&](int e) {
        std::ostringstream x;
        x << "[" << p.net.edge_name[e].q << "," << p.net.edge_name[e].t << "]";
        return x.str();
    };
    o << "{\"n_leaves\":" << p.tree.n_leaves << ",\"lhs\":[";
    for (size_t i = 0; i < p.tree.lhs.size(); ++i) o << (i ? "," : "") << p.tree.lhs[i];
    o << "],\"rhs\":[";
    for (size_t i = 0; i < p.tree.rhs.size(); ++i) o << (i ? "," : "") << p.tree.rhs[i];
    o << "],\"sliced\":[";
    for (size_t i = 0; i < p.sliced.size(); ++i) o << (i ? "," : "") << edge(p.sliced[i]);
    o << "],\"batch_log2\":" << p.batch_log2 << ",\"open\":[";
    for (size_t i = 0; i < p.net.open_edges.size(); ++i) o << (i ? "," : "") << edge(p.net.open_edges[i]);
    o << "],\"leaves\":[";
    for (size_t i = 0; i < p.net.leaves.size(); ++i) {
        o << (i ? "," : "") << "[";
        for (size_t j = 0; j < p.net.leaves[i].legs.size(); ++j)
            o << (j ? "," : "") << edge(p.net.leaves[i].legs[j]);
        o << "]";
    }
    o << "],\"steps\":[";
    for (size_t i = 0; i < p.steps.size(); ++i) {
        const Step& s = p.steps[i];
        o << (i ? "," : "") << "{\"node\":" << s.node << ",\"a\":" << s.a_node << ",\"b\":" << s.b_node
          << ",\"m\":" << s.m_log << ",\"n\":" << s.n_log << ",\"k\":" << s.k_log << ",\"batch\":" << s.b_log
          << ",\"invariant\":" << (s.invariant ? "true" : "false") << ",\"kernel\":" << s.kernel
          << ",\"tile\":" << s.tile << ",\"splitk\":" << s.splitk_log << ",\"cmacs\":" << s.cmacs
          << ",\"bytes\":" << s.bytes;
        // output address bit of each m, n and batch index (C layout)
        auto arr = [&](const char* key, const std::vector<int>& v) {
            o << ",\"" << key << "\":[";
            for (size_t j = 0; j < v.size(); ++j) o << (j ? "," : "") << v[j];
            o << "]";
        };
        arr("c_pos_m", s.c_pos_m);
        arr("c_pos_n", s.c_pos_n);
        arr("c_pos_b", s.c_pos_b);
        o << "}";
    }
    const tn_plan_stats& st = p.stats;
    o << "],\"stats\":{\"n_sliced\":" << st.n_sliced << ",\"batch_log2\":" << st.batch_log2
      << ",\"max_log2_size\":" << st.max_log2_size << ",\"cmacs_per_slice\":" << st.cmacs_per_slice
      << ",\"cmacs_per_slice_unmerged\":" << st.cmacs_per_slice_unmerged
      << ",\"cmacs_per_batch\":" << st.cmacs_per_batch << ",\"bytes_per_batch\":" << st.bytes_per_batch
      << ",\"cmacs_invariant\":" << st.cmacs_invariant << ",\"workspace_bytes\":" << st.workspace_bytes
      << ",\"n_dense_steps\":" << st.n_dense_steps << ",\"n_small_steps\":" << st.n_small_steps << "}}";
    return o.str();
}

}  // namespace tn
