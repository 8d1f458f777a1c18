// Contraction order by hierarchical bipartition (host).
//
// Appendix A, "Finding contraction order using hierarchical partitioning":
// the network is split into two parts recursively; every bipartition is one
// binary node of the contraction tree, and once a part holds few tensors its
// tensors are contracted with a greedy order.  Each bipartition here is a
// min-cut bisection of the tensor graph (one unit of weight per shared bond
// of dimension 2, so the cut size is the number of bits joining the parts,
// the n_AB of Fig. 3) under a size-balance constraint, found from a
// breadth-first initial region refined by Fiduccia-Mattheyses passes.  The
// imbalance, leaf size and seeds are randomised across trials; the planner
// keeps the trial whose sliced cost is lowest.
#include <algorithm>
#include <array>
#include <cmath>
#include <functional>
#include <numeric>
#include <queue>
#include <random>

#include "plan.hpp"

namespace tn {

namespace {

struct Graph {
    // adjacency with multiplicity: adj[v] = list of (u, w)
    std::vector<std::vector<std::pair<int, int>>> adj;
};

// Tensor graph plus one virtual vertex (id L) joined to every open leg with
// weight `open_w`: a cut through open legs is then paid for, so the first
// bisection separates a tail holding the open legs from the head.
Graph leaf_graph(const std::vector<Legs>& leaf_legs, int open_w) {
    const int L = (int)leaf_legs.size();
    int E = 0;
    for (auto& l : leaf_legs)
        for (int e : l) E = std::max(E, e + 1);
    std::vector<std::array<int, 2>> ends(E, {-1, -1});
    for (int i = 0; i < L; ++i)
        for (int e : leaf_legs[i]) (ends[e][0] < 0 ? ends[e][0] : ends[e][1]) = i;
    std::vector<std::vector<std::pair<int, int>>> tmp(L + 1);
    for (int e = 0; e < E; ++e) {
        int a = ends[e][0], b = ends[e][1];
        if (a < 0) continue;
        if (b < 0) {
            if (open_w > 0) {
                tmp[a].push_back({L, open_w});
                tmp[L].push_back({a, open_w});
            }
            continue;
        }
        if (a == b) continue;
        tmp[a].push_back({b, 1});
        tmp[b].push_back({a, 1});
    }
    Graph g;
    g.adj.resize(L + 1);
    for (int v = 0; v <= L; ++v) {   // merge parallel bonds
        auto& t = tmp[v];
        std::sort(t.begin(), t.end());
        for (auto& p : t) {
            if (!g.adj[v].empty() && g.adj[v].back().first == p.first) g.adj[v].back().second += p.second;
            else g.adj[v].push_back(p);
        }
    }
    return g;
}

// Bisect the vertex set `vs` (global ids).  side[v] in {0,1} for v in vs on
// return.  Returns the cut weight.
int bisect(const Graph& g, const std::vector<int>& vs, double eps, std::mt19937_64& rng,
           std::vector<int>& side, std::vector<int>& mark) {
    const int n = (int)vs.size();
    // mark[v] = local index + 1 for members
    for (int i = 0; i < n; ++i) mark[vs[i]] = i + 1;
    const int lo = std::max(1, (int)std::floor(n * (1.0 - eps) / 2.0));
    const int hi = std::min(n - 1, (int)std::ceil(n * (1.0 + eps) / 2.0));
    std::vector<int> best_side;
    int best_cut = -1;
    const int tries = 3;
    for (int t = 0; t < tries; ++t) {
        // initial region: BFS from a random member to n/2 vertices
        std::vector<int> s(n, 1);
        int start = (int)(rng() % n);
        std::vector<char> seen(n, 0);
        std::queue<int> q;
        q.push(start);
        seen[start] = 1;
        int taken = 0;
        const int target = n / 2;
        while (taken < target) {
            if (q.empty()) {   // disconnected: jump to an unseen vertex
                int u = -1;
                for (int i = 0; i < n; ++i)
                    if (!seen[i]) { u = i; break; }
                if (u < 0) break;
                seen[u] = 1;
                q.push(u);
            }
            int u = q.front();
            q.pop();
            s[u] = 0;
            ++taken;
            std::vector<int> nb;
            for (auto& p : g.adj[vs[u]]) {
                int j = mark[p.first] - 1;
                if (j >= 0 && !seen[j]) nb.push_back(j);
            }
            std::shuffle(nb.begin(), nb.end(), rng);
            for (int j : nb) {
                seen[j] = 1;
                q.push(j);
            }
        }
        // FM refinement
        auto cut_of = [&]() {
            int c = 0;
            for (int i = 0; i < n; ++i)
                for (auto& p : g.adj[vs[i]]) {
                    int j = mark[p.first] - 1;
                    if (j > i && s[j] != s[i]) c += p.second;
                }
            return c;
        };
        int cut = cut_of();
        int size0 = 0;
        for (int i = 0; i < n; ++i) size0 += s[i] == 0;
        for (int pass = 0; pass < 12; ++pass) {
            std::vector<int> gain(n, 0);
            for (int i = 0; i < n; ++i)
                for (auto& p : g.adj[vs[i]]) {
                    int j = mark[p.first] - 1;
                    if (j < 0) continue;
                    gain[i] += (s[j] != s[i]) ? p.second : -p.second;
                }
            std::vector<char> locked(n, 0);
            std::vector<int> moved;
            int cur = cut, best = cut, best_len = 0, sz0 = size0;
            for (int step = 0; step < n; ++step) {
                int v = -1, gv = 0;
                for (int i = 0; i < n; ++i) {
                    if (locked[i]) continue;
                    int nsz0 = sz0 + (s[i] == 0 ? -1 : 1);
                    if (nsz0 < lo || nsz0 > hi) continue;
                    if (v < 0 || gain[i] > gv || (gain[i] == gv && (rng() & 1))) {
                        v = i;
                        gv = gain[i];
                    }
                }
                if (v < 0) break;
                locked[v] = 1;
                sz0 += s[v] == 0 ? -1 : 1;
                s[v] ^= 1;
                cur -= gv;
                moved.push_back(v);
                for (auto& p : g.adj[vs[v]]) {
                    int j = mark[p.first] - 1;
                    if (j < 0) continue;
                    // edge (v, j) flipped between cut and uncut
                    if (s[j] == s[v]) gain[j] -= 2 * p.second;
                    else gain[j] += 2 * p.second;
                }
                gain[v] = -gv;
                if (cur < best) {
                    best = cur;
                    best_len = (int)moved.size();
                }
                if ((int)moved.size() - best_len > 50) break;   // no recent improvement
            }
            for (int i = (int)moved.size() - 1; i >= best_len; --i) s[moved[i]] ^= 1;
            size0 = 0;
            for (int i = 0; i < n; ++i) size0 += s[i] == 0;
            if (best >= cut) {
                cut = best;
                break;
            }
            cut = best;
        }
        if (best_cut < 0 || cut < best_cut) {
            best_cut = cut;
            best_side = s;
        }
    }
    for (int i = 0; i < n; ++i) {
        side[vs[i]] = best_side[i];
        mark[vs[i]] = 0;
    }
    return best_cut;
}

}  // namespace

Tree partition_tree(const std::vector<Legs>& leaf_legs, uint64_t seed, double eps, int leaf_size, int open_w,
                    int time_cap, int space_cap) {
    const int L = (int)leaf_legs.size();
    Graph g = leaf_graph(leaf_legs, open_w);
    std::mt19937_64 rng(seed * 0x2545F4914F6CDD1DULL + 99);
    std::vector<int> side(L + 1, 0), mark(L + 1, 0);
    Tree t;
    t.n_leaves = L;
    // legs of a group of leaves: bonds with one end inside (open legs count;
    // the virtual output vertex L is not a leaf)
    auto part_legs = [&](const std::vector<int>& part) {
        Legs all;
        for (int v : part)
            if (v != L) all.insert(all.end(), leaf_legs[v].begin(), leaf_legs[v].end());
        std::sort(all.begin(), all.end());
        Legs out;
        for (size_t i = 0; i < all.size();) {
            size_t j = i;
            while (j < all.size() && all[j] == all[i]) ++j;
            if (j - i == 1) out.push_back(all[i]);
            i = j;
        }
        return out;
    };
    // recursive bisection, emitting steps bottom-up; the virtual output
    // vertex L takes part in the cuts but is never contracted
    std::function<int(std::vector<int>)> rec = [&](std::vector<int> vs) -> int {
        std::vector<int> real;
        for (int v : vs)
            if (v != L) real.push_back(v);
        if (real.empty()) return -1;
        if (real.size() == 1) return real[0];
        if ((int)real.size() <= leaf_size) vs = real;
        if ((int)vs.size() <= leaf_size) {
            std::vector<Legs> sub;
            for (int v : vs) sub.push_back(leaf_legs[v]);
            Tree st = greedy_tree(sub, rng(), 1.0, 0.0);
            std::vector<int> id(st.n_nodes());
            for (int i = 0; i < st.n_leaves; ++i) id[i] = vs[i];
            for (size_t s = 0; s < st.lhs.size(); ++s) {
                int a = id[st.lhs[s]], b = id[st.rhs[s]];
                t.lhs.push_back(a);
                t.rhs.push_back(b);
                id[st.n_leaves + s] = L + (int)t.lhs.size() - 1;
            }
            return id[st.n_nodes() - 1];
        }
        std::vector<int> a, b;
        if (time_cap <= 0 && space_cap <= 0) {
            bisect(g, vs, eps, rng, side, mark);
            for (int v : vs) (side[v] == 0 ? a : b).push_back(v);
        } else {
            // time and space caps on this bisection's own contraction:
            // retry with other imbalances until within both caps (or keep
            // the split with the smallest excess, then the smallest cut)
            int best_excess = -1, best_cut = 0;
            for (int tr = 0; tr < 6; ++tr) {
                const double e = tr == 0 ? eps : std::min(0.9, eps * (1.0 + 0.5 * tr));
                const int cut = bisect(g, vs, e, rng, side, mark);
                std::vector<int> ta, tb;
                for (int v : vs) (side[v] == 0 ? ta : tb).push_back(v);
                const Legs la = part_legs(ta), lb = part_legs(tb);
                const int u = (int)set_union(la, lb).size(), o = (int)set_xor(la, lb).size();
                const int excess = (time_cap > 0 ? std::max(0, u - time_cap) : 0) +
                                   (space_cap > 0 ? std::max(0, o - space_cap) : 0);
                if (best_excess < 0 || excess < best_excess || (excess == best_excess && cut < best_cut)) {
                    best_excess = excess;
                    best_cut = cut;
                    a = ta;
                    b = tb;
                }
                if (excess == 0) break;
            }
        }
        if (a.empty() || b.empty()) {   // degenerate split: halve by order
            a.assign(vs.begin(), vs.begin() + vs.size() / 2);
            b.assign(vs.begin() + vs.size() / 2, vs.end());
        }
        int ra = rec(a);
        int rb = rec(b);
        if (ra < 0) return rb;
        if (rb < 0) return ra;
        t.lhs.push_back(ra);
        t.rhs.push_back(rb);
        return L + (int)t.lhs.size() - 1;
    };
    std::vector<int> all(L + (open_w > 0 ? 1 : 0));
    std::iota(all.begin(), all.end(), 0);
    if (L > 1) rec(all);
    return t;
}

}  // namespace tn
