// Canonical tensor network of a circuit (host).
//
// Section "Computing bitstring probabilities": single-qubit gates are
// absorbed into two-qubit gates, giving one node per two-qubit gate.  The
// rules fixed here (and restated in tn.h): absorption runs forward into the
// next two-qubit gate on the qubit, trailing single-qubit gates go backward
// into the last one, |0> is absorbed into a qubit's first two-qubit gate and
// the projector <s1_q| of a closed qubit into its last one; edge (q, t) is
// the wire of qubit q after its t-th two-qubit gate.
#include <algorithm>
#include <array>
#include <map>
#include <set>

#include "plan.hpp"

namespace tn {

namespace {

struct NamedTensor {
    std::vector<EdgeName> names;   // names[i] <-> address bit i
    std::vector<cd> data;
};

// Fix bit `bit` of the tensor to value v and drop that leg.
void take(NamedTensor& t, int bit, int v) {
    const size_t n = t.data.size() / 2;
    std::vector<cd> out(n);
    const size_t lo_mask = (size_t(1) << bit) - 1;
    for (size_t i = 0; i < n; ++i) {
        size_t lo = i & lo_mask;
        size_t old = ((i - lo) << 1) | (size_t(v) << bit) | lo;
        out[i] = t.data[old];
    }
    t.data.swap(out);
    t.names.erase(t.names.begin() + bit);
}

// new[.., a, ..] = sum_b m[a][b] old[.., b, ..] on leg `bit`.
void apply2(NamedTensor& t, int bit, const cd m[2][2]) {
    const size_t stride = size_t(1) << bit;
    std::vector<cd> out(t.data.size());
    for (size_t i = 0; i < t.data.size(); ++i) {
        int a = (i >> bit) & 1;
        size_t i0 = i & ~stride, i1 = i | stride;
        out[i] = m[a][0] * t.data[i0] + m[a][1] * t.data[i1];
    }
    t.data.swap(out);
}

void matmul2(const cd a[2][2], const cd b[2][2], cd out[2][2]) {
    cd r[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) r[i][j] = a[i][0] * b[0][j] + a[i][1] * b[1][j];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) out[i][j] = r[i][j];
}

void set_identity(cd m[2][2]) {
    m[0][0] = 1; m[0][1] = 0; m[1][0] = 0; m[1][1] = 1;
}

}  // namespace

int Network::find_edge(int q, int t) const {
    for (size_t e = 0; e < edge_name.size(); ++e)
        if (edge_name[e].q == q && edge_name[e].t == t) return (int)e;
    return -1;
}

std::string build_network(const tn_circuit& c, const std::vector<int>& open_q,
                          const std::vector<int>& fixed_q, const std::vector<uint8_t>& bits,
                          Network& out) {
    const int n = c.n_qubits;
    if (n <= 0 || n > 4096) return "n_qubits out of range";
    if (c.n_gates < 0 || (c.n_gates > 0 && !c.gates)) return "bad gate list";
    std::vector<int> role(n, -1);   // 0 open, 1 fixed
    std::vector<int> bit_of(n, 0);
    for (int q : open_q) {
        if (q < 0 || q >= n || role[q] != -1) return "open qubits: out of range or repeated";
        role[q] = 0;
    }
    for (size_t i = 0; i < fixed_q.size(); ++i) {
        int q = fixed_q[i];
        if (q < 0 || q >= n || role[q] != -1) return "fixed qubits: out of range or overlapping";
        if (bits[i] > 1) return "fixed bits must be 0 or 1";
        role[q] = 1;
        bit_of[q] = bits[i];
    }
    for (int q = 0; q < n; ++q)
        if (role[q] == -1) return "every qubit must be open or fixed";

    std::vector<std::array<std::array<cd, 2>, 2>> pend(n);
    auto pend_ptr = [&](int q) { return reinterpret_cast<cd(*)[2]>(pend[q].data()); };
    for (int q = 0; q < n; ++q) set_identity(pend_ptr(q));
    std::vector<int> count(n, 0), holder(n, -1);
    std::vector<NamedTensor> ts;

    for (int g = 0; g < c.n_gates; ++g) {
        const tn_gate& G = c.gates[g];
        if (G.q0 < 0 || G.q0 >= n || G.q1 >= n || G.q1 < -1 || G.q1 == G.q0)
            return "gate " + std::to_string(g) + ": bad qubits";
        if (G.q1 < 0) {
            cd m[2][2] = {{cd(G.re[0], G.im[0]), cd(G.re[1], G.im[1])},
                          {cd(G.re[2], G.im[2]), cd(G.re[3], G.im[3])}};
            matmul2(m, pend_ptr(G.q0), pend_ptr(G.q0));
            continue;
        }
        const int q0 = G.q0, q1 = G.q1;
        // U = M (P0 (x) P1)
        cd U[4][4];
        auto P0 = pend_ptr(q0);
        auto P1 = pend_ptr(q1);
        for (int r = 0; r < 4; ++r)
            for (int col = 0; col < 4; ++col) {
                cd acc = 0;
                int ci = col >> 1, cj = col & 1;
                for (int k = 0; k < 4; ++k) {
                    int ki = k >> 1, kj = k & 1;
                    acc += cd(G.re[4 * r + k], G.im[4 * r + k]) * P0[ki][ci] * P1[kj][cj];
                }
                U[r][col] = acc;
            }
        set_identity(P0);
        set_identity(P1);
        NamedTensor t;
        t.names = {{q0, count[q0]}, {q1, count[q1]}, {q0, count[q0] - 1}, {q1, count[q1] - 1}};
        t.data.resize(16);
        for (int idx = 0; idx < 16; ++idx) {
            int o0 = idx & 1, o1 = (idx >> 1) & 1, i0 = (idx >> 2) & 1, i1 = (idx >> 3) & 1;
            t.data[idx] = U[2 * o0 + o1][2 * i0 + i1];
        }
        if (count[q1] == 0) take(t, 3, 0);   // |0> on q1
        if (count[q0] == 0) take(t, 2, 0);   // |0> on q0
        ts.push_back(std::move(t));
        holder[q0] = holder[q1] = (int)ts.size() - 1;
        count[q0]++;
        count[q1]++;
    }
    // trailing single-qubit gates, projectors, gate-less qubits
    for (int q = 0; q < n; ++q) {
        if (count[q] == 0) {
            auto P = pend_ptr(q);
            NamedTensor t;
            t.names = {{q, -1}};
            t.data = {P[0][0], P[1][0]};
            if (role[q] == 1) take(t, 0, bit_of[q]);
            ts.push_back(std::move(t));
            continue;
        }
        NamedTensor& t = ts[holder[q]];
        EdgeName nm{q, count[q] - 1};
        int bit = -1;
        for (size_t i = 0; i < t.names.size(); ++i)
            if (t.names[i] == nm) bit = (int)i;
        if (bit < 0) return "internal error: lost out-leg";
        apply2(t, bit, pend_ptr(q));
        if (role[q] == 1) take(t, bit, bit_of[q]);
    }
    // canonical edge ids: sorted names
    std::set<EdgeName> names;
    for (auto& t : ts)
        for (auto& nm : t.names) names.insert(nm);
    std::map<EdgeName, int> id;
    out = Network();
    out.n_qubits = n;
    for (auto& nm : names) {
        id[nm] = (int)out.edge_name.size();
        out.edge_name.push_back(nm);
        out.end0.push_back(-1);
        out.end1.push_back(-1);
    }
    for (size_t li = 0; li < ts.size(); ++li) {
        HostTensor h;
        for (auto& nm : ts[li].names) {
            int e = id[nm];
            h.legs.push_back(e);
            if (out.end0[e] < 0) out.end0[e] = (int)li;
            else out.end1[e] = (int)li;
        }
        h.data = std::move(ts[li].data);
        out.leaves.push_back(std::move(h));
    }
    std::vector<int> sorted_open = open_q;
    std::sort(sorted_open.begin(), sorted_open.end());
    for (int q : sorted_open) {
        EdgeName nm{q, count[q] > 0 ? count[q] - 1 : -1};
        auto it = id.find(nm);
        if (it == id.end()) return "internal error: missing open leg";
        out.open_edges.push_back(it->second);
    }
    std::vector<char> is_open(out.edge_name.size(), 0);
    for (int e : out.open_edges) is_open[e] = 1;
    for (size_t e = 0; e < out.edge_name.size(); ++e) {
        bool two = out.end1[e] >= 0;
        if (is_open[e] == two) return "internal error: edge ends";
    }
    return "";
}

}  // namespace tn
