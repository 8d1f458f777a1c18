// Executor: uploads a plan's leaves, computes its slice-invariant subtrees
// once, then runs the slice-dependent steps of each launch group (2^b slices
// whose batch legs are contracted together) followed by the float64 slice
// sum ("summation of the final tensors", appendix B).
#include "exec.hpp"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <cstdio>
#include <map>

#include "tiles.hpp"

namespace tn {

std::string run_groups_eager(Plan& p, DeviceState& d, void* ws, double* acc, const std::vector<Group>& groups,
                             hipStream_t s);

namespace {

#define TN_HIP(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) return std::string(#call) + ": " + hipGetErrorString(e_); \
    } while (0)

void put_leaf(const HostTensor& h, const std::vector<int>& layout, int storage, unsigned char* dst) {
    const size_t r = layout.size();
    std::vector<int> src_bit(r);
    for (size_t j = 0; j < r; ++j) {
        auto it = std::find(h.legs.begin(), h.legs.end(), layout[j]);
        src_bit[j] = (int)(it - h.legs.begin());
    }
    const size_t n = size_t(1) << r;
    for (size_t x = 0; x < n; ++x) {
        size_t old = 0;
        for (size_t j = 0; j < r; ++j) old |= ((x >> j) & 1) << src_bit[j];
        const cd v = h.data[old];
        if (storage == ST_C128) {
            double t[2] = {v.real(), v.imag()};
            std::memcpy(dst + 16 * x, t, 16);
        } else {
            float t[2] = {(float)v.real(), (float)v.imag()};
            std::memcpy(dst + 8 * x, t, 8);
        }
    }
}

void* node_ptr(const Plan& p, const DeviceState& d, void* ws, int node, uint64_t slice_base) {
    const NodeInfo& ni = p.nodes[node];
    unsigned char* base = ni.home == HOME_WS ? (unsigned char*)ws : (unsigned char*)d.plan_mem;
    uint64_t off = ni.off;
    if (ni.home == HOME_LEAF && !ni.sliced_bits.empty()) {
        const int lo = (int)ni.layout.size() - (int)ni.sliced_bits.size();
        for (size_t i = 0; i < ni.sliced_bits.size(); ++i)
            off += ((slice_base >> ni.sliced_bits[i]) & 1ull) << (lo + (int)i);
    }
    return base + off * (uint64_t)p.esize;
}

int lp_mode(tn_precision p) {
    switch (p) {
        case TN_SPLIT_FP16: return LP_SPLIT_FP16;
        case TN_BF16: return LP_BF16;
        default: return -1;
    }
}

// Slice selection of a leaf read from device memory (graph replays).
int leaf_select(const Plan& p, int node, uint8_t* bit, uint8_t* pos) {
    const NodeInfo& ni = p.nodes[node];
    if (ni.home != HOME_LEAF || ni.sliced_bits.empty()) return 0;
    const int lo = (int)ni.layout.size() - (int)ni.sliced_bits.size();
    const int n = std::min<int>(8, (int)ni.sliced_bits.size());
    for (int i = 0; i < n; ++i) {
        bit[i] = (uint8_t)ni.sliced_bits[i];
        pos[i] = (uint8_t)(lo + i);
    }
    return n;
}

// always_max: write the output's max-magnitude slot whatever kernel consumes
// it (slice-invariant tensors are computed once, before autotuning or a forced
// configuration may move their consumer to a low-precision MFMA kernel).
std::string launch_step(const Plan& p, const DeviceState& d, const Step& st, const void* A, const void* B, void* C,
                        void* ws, hipStream_t s, std::string* name = nullptr, const uint64_t* d_slice = nullptr,
                        bool always_max = false) {
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    g.A = A;
    g.B = B;
    g.C = C;
    if (d_slice) {
        g.d_slice = d_slice;
        g.sa_n = (uint8_t)leaf_select(p, st.a_node, g.sa_bit, g.sa_pos);
        g.sb_n = (uint8_t)leaf_select(p, st.b_node, g.sb_bit, g.sb_pos);
        if (g.sa_n == 0 && g.sb_n == 0) g.d_slice = nullptr;
    }
    if (d.d_max) {
        g.amax = d.d_max + p.nodes[st.a_node].slot;
        g.bmax = d.d_max + p.nodes[st.b_node].slot;
        // the output's max is needed only when a low-precision MFMA step
        // (tiled or panel) consumes it
        const int parent = p.nodes[st.node].parent;
        if (parent >= 0 && p.step_of_node[parent] >= 0) {
            const int ck = p.steps[p.step_of_node[parent]].kernel;
            if (always_max || ck == K_MFMA || ck == K_PANEL) g.cmax = d.d_max + p.nodes[st.node].slot;
        }
    }
    const int mode = lp_mode(p.opts.prec);
    g.m_log = st.m_log;
    g.n_log = st.n_log;
    g.k_log = st.k_log;
    g.b_log = st.b_log;
    if (st.m_log > kMaxBits || st.n_log > kMaxBits || st.b_log > kMaxBits) return "step too large";
    for (int i = 0; i < st.m_log; ++i) g.cpm[i] = (uint8_t)st.c_pos_m[i];
    for (int i = 0; i < st.n_log; ++i) g.cpn[i] = (uint8_t)st.c_pos_n[i];
    for (int i = 0; i < st.b_log; ++i) g.cpb[i] = (uint8_t)st.c_pos_b[i];
    const int storage = storage_of(p.opts.prec);
    const size_t esz = storage == ST_C128 ? 16 : 8;
    int R = 1;
    if (st.kernel == K_MFMA) {
        g.tm = kMfmaTiles[st.tile].tm_log;
        g.tn = kMfmaTiles[st.tile].tn_log;
        g.tk = std::min(kMfmaTiles[st.tile].tk_max_log, st.k_log);
    } else if (st.kernel == K_STREAM) {
        g.tm = g.tn = g.tk = 0;
    } else if (st.kernel == K_SKINNY) {
        g.tm = 5;   // each wave stages 32 rows x 16 columns of C at a time
        g.tn = 4;
        g.tk = st.k_log;
    } else if (st.kernel == K_PANEL) {
        g.tm = 7;   // the block stages 128 rows x 16 columns of C at a time
        g.tn = 4;   // (the epilogue decode); the tile width is set below
        g.tk = panel_kc_log(st.tile);
    } else {
        const int m = st.m_log, n = st.n_log;
        g.split_log = st.kernel == K_SPLITK ? st.splitk_log : 0;
        const int k = st.k_log - g.split_log;
        const int r_log = (m + n >= 10) ? 2 : (m + n >= 9 ? 1 : 0);
        const int tile_log = std::min(8 + r_log, m + n);
        // keep all of a small N in the tile (else A is re-read once per
        // N-tile), give M the rest, then any remainder back to N
        g.tn = std::min(n, std::min(4, tile_log));
        g.tm = std::min(m, tile_log - g.tn);
        g.tn = std::min(n, tile_log - g.tm);
        R = 1 << std::max(0, g.tm + g.tn - 8);
        const int limit = (int)(32768 / esz);
        int tk = 0;
        while (tk < k && (2 << tk) * ((1 << g.tm) + (1 << g.tn)) <= limit) ++tk;
        g.tk = tk;
        if (g.split_log > 0) g.scratch = (unsigned char*)ws + st.scratch_off * (uint64_t)p.esize;
    }
    if (st.kernel == K_STREAM) {
        if (name) *name = storage == ST_C128 ? "k_stream<double2,1>" : "k_stream<float2,2>";
        hipError_t e = launch_stream(storage, g, s);
        if (e != hipSuccess) return std::string("stream launch: ") + hipGetErrorString(e);
        return "";
    }
    // epilogue decode: tile bits of C sorted by address position
    std::vector<std::pair<int, int>> ep;
    for (int i = 0; i < g.tm; ++i) ep.push_back({st.c_pos_m[i], i});
    for (int j = 0; j < g.tn; ++j) ep.push_back({st.c_pos_n[j], 32 + j});
    std::sort(ep.begin(), ep.end());
    if (ep.size() > 16) return "epilogue tile too large";
    g.ep_n = (int)ep.size();
    for (size_t i = 0; i < ep.size(); ++i) {
        g.ep_pos[i] = (uint8_t)ep[i].first;
        g.ep_src[i] = (uint8_t)ep[i].second;
    }
    if (st.kernel == K_PANEL) {
        g.tn = panel_tn_log(st.tile);
        // names as profilers show the device functions (template arguments)
        const int tnl = panel_tn_log(st.tile);
        const std::string kcnb = std::string(panel_kc_log(st.tile) == 5 ? "32," : "16,") +
                                 (tnl == 7 ? "8," : (tnl == 6 ? "4," : "2,"));
        const bool nt = st.tile & 16;
        hipError_t e;
        if (!panel_fp32(st.tile, p.opts.prec)) {
            // tile bit 3: split A in registers inside the GEMM (no pass over A)
            uint32_t* conv = (ws && st.conv_off != ~uint64_t(0) && !(st.tile & 8))
                                 ? reinterpret_cast<uint32_t*>((unsigned char*)ws + st.conv_off * (uint64_t)p.esize)
                                 : nullptr;
            const int lt = conv ? (st.tile & 67) : (st.tile & 83);
            if (name)
                *name = std::string(conv ? "k_lp_convert_a+" : "") + "k_panel_lp<" + kcnb + std::to_string(mode) +
                        (conv ? ",true," : ",false,") + (!conv && nt ? "true>" : "false>");
            e = launch_panel_lp(mode, lt, g, conv, s);
        } else {
            const bool three = st.tile & 32;
            if (name)
                *name = (st.tile & 128) ? std::string("k_panel3d<") + (tnl == 6 ? "4>" : "2>")
                                        : std::string(three ? "k_panel3<" : "k_panel<") + kcnb + (nt ? "true>" : "false>");
            e = launch_panel(st.tile & 179, g, s);
        }
        if (e != hipSuccess) return std::string("panel launch: ") + hipGetErrorString(e);
        return "";
    }
    if (st.kernel == K_SKINNY) {
        if (name)
            *name = "k_skinny<" + std::to_string(1 << std::min(st.k_log, 6)) + "," +
                    std::to_string(1 << std::max(0, st.n_log - 4)) + ">";
        hipError_t e = launch_skinny(g, s);
        if (e != hipSuccess) return std::string("skinny launch: ") + hipGetErrorString(e);
        return "";
    }
    if (name) {
        static const char* tile_names[] = {"<4,4,2,2", "<2,2,2,2", "<2,2,4,1", "<1,1,4,1", "<4,1,4,1"};
        static const char* mode_names[] = {",0>", ",1>", ",2>"};
        if (st.kernel == K_MFMA)
            *name = mode < 0 ? std::string("k_mfma_c64") + tile_names[st.tile] + ">"
                             : std::string("k_mfma_lp") + tile_names[st.tile] + mode_names[mode];
        else *name = std::string("k_valu<") + (storage == ST_C128 ? "double2," : "float2,") + std::to_string(R) +
                     ">" + (g.split_log > 0 ? "+k_splitk_red" : "");
    }
    hipError_t e;
    if (st.kernel == K_MFMA) {
        e = launch_mfma(mode, st.tile, g, s);
    } else {
        e = launch_valu(storage, g, R, s);
        if (e == hipSuccess && g.split_log > 0) e = launch_splitk_reduce(storage, g, s);
    }
    if (e != hipSuccess) return std::string("step launch: ") + hipGetErrorString(e);
    return "";
}

std::string profile_harvest_set(DeviceState& d, int set) {
    Profiler& pf = d.prof;
    if (!pf.pending[set]) return "";
    const int n = (int)pf.ms.size();
    TN_HIP(hipEventSynchronize(pf.ev[set][n]));
    for (int i = 0; i < n; ++i) {
        float ms = 0.f;
        TN_HIP(hipEventElapsedTime(&ms, pf.ev[set][i], pf.ev[set][i + 1]));
        pf.ms[i] += ms;
        pf.launches[i] += 1;
    }
    pf.pending[set] = false;
    return "";
}

}  // namespace

// Destroy the captured graph once every replay queued from it has finished:
// its kernel nodes' argument buffers belong to the executable graph.
static std::string drop_graph(DeviceState& d, int which) {
    if (!d.gexec[which]) return "";
    hipError_t e = d.g_done ? hipEventSynchronize(d.g_done) : hipSuccess;
    (void)hipGraphExecDestroy(d.gexec[which]);
    d.gexec[which] = nullptr;
    if (e != hipSuccess) return std::string("hipEventSynchronize: ") + hipGetErrorString(e);
    return "";
}

static std::string drop_graphs(DeviceState& d) {
    std::string e = drop_graph(d, 0);
    std::string e1 = drop_graph(d, 1);
    for (auto& ln : d.lanes) {
        std::string el = drop_graphs(ln->d);
        if (e1.empty()) e1 = el;
    }
    return e.empty() ? e1 : e;
}

std::string profile_harvest(DeviceState& d) {
    std::string e = profile_harvest_set(d, 0);
    if (!e.empty()) return e;
    return profile_harvest_set(d, 1);
}

std::string profile_enable(Plan& p, DeviceState& d, bool on) {
    Profiler& pf = d.prof;
    if (pf.on) {
        std::string e = profile_harvest(d);
        if (!e.empty()) return e;
    }
    const int n = (int)p.steps.size() - p.n_invariant_steps + 1;
    if (on) {
        for (int set = 0; set < 2; ++set) {
            if ((int)pf.ev[set].size() != n + 1) {
                for (auto ev : pf.ev[set]) (void)hipEventDestroy(ev);
                pf.ev[set].assign(n + 1, nullptr);
                for (auto& ev : pf.ev[set]) TN_HIP(hipEventCreate(&ev));
            }
            pf.pending[set] = false;
        }
        pf.ms.assign(n, 0.0);
        pf.launches.assign(n, 0);
        pf.names.assign(n, std::string());
    }
    pf.on = on;
    return "";
}

int storage_of(tn_precision p) {
    switch (p) {
        case TN_C128: return ST_C128;
        default: return ST_C64;   // split-FP16 and BF16 keep complex64 storage
    }
}

std::string prepare(Plan& p, DeviceState& d, hipStream_t s) {
    int dev = 0;
    TN_HIP(hipGetDevice(&dev));
    if (d.prepared && d.device == dev) return "";
    if (d.prepared && d.device != dev) return "plan was prepared on another device";
    const int storage = storage_of(p.opts.prec);
    d.device = dev;
    d.plan_bytes = std::max<uint64_t>(p.plan_elems, 64) * (uint64_t)p.esize;
    TN_HIP(hipMalloc(&d.plan_mem, d.plan_bytes));
    std::vector<unsigned char> host(d.plan_bytes, 0);
    for (int i = 0; i < p.tree.n_leaves; ++i)
        put_leaf(p.net.leaves[i], p.nodes[i].layout, storage, host.data() + p.nodes[i].off * p.esize);
    TN_HIP(hipMemcpy(d.plan_mem, host.data(), d.plan_bytes, hipMemcpyHostToDevice));
    if (lp_mode(p.opts.prec) >= 0) {
        // max-magnitude slots: leaves from the host data, the rest zero
        const int n_slots = (int)p.tree.n_nodes();
        std::vector<float> h(n_slots, 0.f);
        for (int i = 0; i < p.tree.n_leaves; ++i) {
            double m = 0;
            for (const cd& v : p.net.leaves[i].data) m = std::max(m, std::max(std::abs(v.real()), std::abs(v.imag())));
            h[p.nodes[i].slot] = (float)m;
        }
        TN_HIP(hipMalloc(&d.d_max, sizeof(float) * n_slots));
        TN_HIP(hipMemcpy(d.d_max, h.data(), sizeof(float) * n_slots, hipMemcpyHostToDevice));
    }
    for (const Step& st : p.steps) {
        if (!st.invariant) continue;
        void* A = node_ptr(p, d, nullptr, st.a_node, 0);
        void* B = node_ptr(p, d, nullptr, st.b_node, 0);
        void* C = (unsigned char*)d.plan_mem + st.c_off * (uint64_t)p.esize;
        if (st.kernel == K_SPLITK) return "split-K step in the slice-invariant part needs a workspace";
        std::string err = launch_step(p, d, st, A, B, C, nullptr, s, nullptr, nullptr, true);
        if (!err.empty()) return err;
    }
    d.mask_words = std::max<size_t>(1, ((size_t(1) << p.batch_log2) + 31) / 32);
    TN_HIP(hipMalloc(&d.d_state, sizeof(GroupState)));
    TN_HIP(hipMemset(d.d_state, 0, sizeof(GroupState)));
    TN_HIP(hipStreamSynchronize(s));
    d.prepared = true;
    return "";
}

std::string upload_leaf(Plan& p, DeviceState& d, int leaf, std::vector<cd> data, hipStream_t s) {
    if (!d.prepared) return "plan not prepared";
    if (leaf < 0 || leaf >= p.tree.n_leaves) return "leaf out of range";
    const size_t n = size_t(1) << p.nodes[leaf].layout.size();
    if (data.size() != n || p.net.leaves[leaf].data.size() != n) return "leaf data size mismatch";
    HostTensor h;
    h.legs = p.net.leaves[leaf].legs;
    h.data = std::move(data);
    std::vector<unsigned char> host(n * (size_t)p.esize);
    put_leaf(h, p.nodes[leaf].layout, storage_of(p.opts.prec), host.data());
    TN_HIP(hipMemcpyAsync((unsigned char*)d.plan_mem + p.nodes[leaf].off * (uint64_t)p.esize, host.data(), host.size(),
                          hipMemcpyHostToDevice, s));
    TN_HIP(hipStreamSynchronize(s));   // the host buffer ends here
    return "";
}

// Launch groups captured in one graph: enough to cover a bench step of 4096
// slices at 2^8 slices per group, with at most about 4096 kernel nodes.
constexpr int kMaxGraphGroups = 16;
constexpr int kMaxGraphNodes = 4096;

static int many_groups(const Plan& p) {
    const int per_group = (int)p.steps.size() - p.n_invariant_steps + 3;
    int g = 1;
    while (g * 2 <= kMaxGraphGroups && g * 2 * per_group <= kMaxGraphNodes) g *= 2;
    return g;
}

// Capture n_groups full launch groups (slice id read from device memory)
// into one graph: per group, group-begin (advances the group index), max-slot
// reset, every slice-dependent step, slice sum.
static std::string build_graph(Plan& p, DeviceState& d, void* ws, double* acc, int which, int n_groups) {
    std::string derr = drop_graph(d, which);
    if (!derr.empty()) return derr;
    if (!d.cap_stream) TN_HIP(hipStreamCreateWithFlags(&d.cap_stream, hipStreamNonBlocking));
    const int storage = storage_of(p.opts.prec);
    hipStream_t c = d.cap_stream;
    const uint64_t* dsl = &d.d_state->slice_base;
    TN_HIP(hipStreamBeginCapture(c, hipStreamCaptureModeThreadLocal));
    std::string err;
    for (int gi = 0; gi < n_groups && err.empty(); ++gi) {
        hipError_t e = launch_group_begin(d.d_state, p.batch_log2, c);
        if (e == hipSuccess && d.d_max)
            e = launch_fill(d.d_max + p.n_static_slots, (uint64_t)(p.tree.n_nodes() - p.n_static_slots), c);
        if (e != hipSuccess) err = std::string("graph: ") + hipGetErrorString(e);
        for (const Step& st : p.steps) {
            if (!err.empty()) break;
            if (st.invariant) continue;
            void* A = node_ptr(p, d, ws, st.a_node, 0);
            void* B = node_ptr(p, d, ws, st.b_node, 0);
            void* C = (unsigned char*)ws + st.c_off * (uint64_t)p.esize;
            err = launch_step(p, d, st, A, B, C, ws, c, nullptr, dsl);
        }
        if (err.empty()) {
            const int root = p.tree.root();
            uint8_t bit[8], pos[8];
            const int rn = leaf_select(p, root, bit, pos);
            e = launch_slice_sum(storage, node_ptr(p, d, ws, root, 0), acc, p.root_log2, p.batch_log2, nullptr, 0,
                                 1ull << p.batch_log2, c, rn ? dsl : nullptr, bit, pos, rn);
            if (e != hipSuccess) err = std::string("graph slice sum: ") + hipGetErrorString(e);
        }
    }
    hipGraph_t graph = nullptr;
    hipError_t ee = hipStreamEndCapture(c, &graph);
    if (err.empty() && ee != hipSuccess) err = std::string("hipStreamEndCapture: ") + hipGetErrorString(ee);
    if (err.empty()) {
        ee = hipGraphInstantiate(&d.gexec[which], graph, nullptr, nullptr, 0);
        if (ee != hipSuccess) err = std::string("hipGraphInstantiate: ") + hipGetErrorString(ee);
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (err.empty()) {
        d.g_ws[which] = ws;
        d.g_acc[which] = acc;
        if (which == 1) d.g_many = n_groups;
    } else {
        d.gexec[which] = nullptr;
    }
    return err;
}

std::string run_groups(Plan& p, DeviceState& d, void* ws, double* acc, const std::vector<Group>& groups,
                       hipStream_t s) {
    // runs of full, consecutive launch groups are replayed from captured
    // graphs (several groups per launch where the run is long enough) unless
    // per-step timing is on (it needs eager launches)
    static const bool no_graph = std::getenv("TN_NO_GRAPH") != nullptr;
    if (!d.prof.on && !no_graph && d.d_state && groups.size() >= 2) {
        size_t i = 0;
        std::vector<Group> eager;
        const int many = many_groups(p);
        while (i < groups.size()) {
            size_t j = i;
            const uint64_t B = 1ull << p.batch_log2;
            while (j < groups.size() && groups[j].mask.empty() && groups[j].beta0 == 0 && groups[j].beta1 == B &&
                   groups[j].slice_base == groups[i].slice_base + ((uint64_t)(j - i) << p.batch_log2))
                ++j;
            if (j - i >= 2) {
                if (!eager.empty()) {
                    std::string e = run_groups_eager(p, d, ws, acc, eager, s);
                    if (!e.empty()) return e;
                    eager.clear();
                }
                const size_t n = j - i;
                const size_t n_many = many > 1 ? n / (size_t)many : 0;
                const size_t n_one = n - n_many * (size_t)many;
                if (n_many && (!d.gexec[1] || d.g_ws[1] != ws || d.g_acc[1] != acc || d.g_many != many)) {
                    std::string e = build_graph(p, d, ws, acc, 1, many);
                    if (!e.empty()) return e;
                }
                if (n_one && (!d.gexec[0] || d.g_ws[0] != ws || d.g_acc[0] != acc)) {
                    std::string e = build_graph(p, d, ws, acc, 0, 1);
                    if (!e.empty()) return e;
                }
                TN_HIP(launch_group_set(d.d_state, groups[i].slice_base >> p.batch_log2, s));
                for (size_t k = 0; k < n_many; ++k) TN_HIP(hipGraphLaunch(d.gexec[1], s));
                for (size_t k = 0; k < n_one; ++k) TN_HIP(hipGraphLaunch(d.gexec[0], s));
                if (!d.g_done) TN_HIP(hipEventCreateWithFlags(&d.g_done, hipEventDisableTiming));
                TN_HIP(hipEventRecord(d.g_done, s));
                d.graph_replays += n;
                d.graph_launches += n_many + n_one;
                i = j;
            } else {
                eager.push_back(groups[i]);
                ++i;
            }
        }
        if (!eager.empty()) return run_groups_eager(p, d, ws, acc, eager, s);
        return "";
    }
    return run_groups_eager(p, d, ws, acc, groups, s);
}

std::string run_groups_eager(Plan& p, DeviceState& d, void* ws, double* acc, const std::vector<Group>& groups,
                             hipStream_t s) {
    const int storage = storage_of(p.opts.prec);
    const int root = p.tree.root();
    // explicit masks: upload all of them first (blocking), then launch
    std::vector<size_t> mask_slot(groups.size(), (size_t)-1);
    size_t n_masks = 0;
    for (size_t i = 0; i < groups.size(); ++i)
        if (!groups[i].mask.empty()) mask_slot[i] = n_masks++;
    uint32_t* d_masks = nullptr;
    if (n_masks) {
        std::vector<uint32_t> h(n_masks * d.mask_words, 0);
        for (size_t i = 0; i < groups.size(); ++i)
            if (mask_slot[i] != (size_t)-1)
                std::copy(groups[i].mask.begin(), groups[i].mask.end(), h.begin() + mask_slot[i] * d.mask_words);
        TN_HIP(hipMallocAsync((void**)&d_masks, h.size() * 4, s));
        TN_HIP(hipMemcpyAsync(d_masks, h.data(), h.size() * 4, hipMemcpyHostToDevice, s));
        TN_HIP(hipStreamSynchronize(s));
    }
    std::string err;
    Profiler& pf = d.prof;
    const int n_dep = (int)p.steps.size() - p.n_invariant_steps;
    if (pf.on && pf.ms.size() != (size_t)n_dep + 1) return "profiler not sized for this plan";
    for (size_t gi = 0; gi < groups.size() && err.empty(); ++gi) {
        const Group& G = groups[gi];
        const int set = (int)(gi & 1);
        if (pf.on) {
            if (pf.pending[set]) {   // harvest the group queued two groups ago
                err = profile_harvest_set(d, set);
                if (!err.empty()) break;
            }
            TN_HIP(hipEventRecord(pf.ev[set][0], s));
        }
        if (d.d_max) {   // reset the max slots of this group's tensors
            const int n_slots = p.tree.n_nodes();
            hipError_t e = launch_fill(d.d_max + p.n_static_slots, (uint64_t)(n_slots - p.n_static_slots), s);
            if (e != hipSuccess) {
                err = std::string("fill: ") + hipGetErrorString(e);
                break;
            }
        }
        int di = 0;
        for (const Step& st : p.steps) {
            if (st.invariant) continue;
            void* A = node_ptr(p, d, ws, st.a_node, G.slice_base);
            void* B = node_ptr(p, d, ws, st.b_node, G.slice_base);
            void* C = (unsigned char*)ws + st.c_off * (uint64_t)p.esize;
            std::string nm;
            err = launch_step(p, d, st, A, B, C, ws, s, pf.on && pf.names[di].empty() ? &nm : nullptr);
            if (!err.empty()) break;
            if (pf.on) {
                if (!nm.empty()) pf.names[di] = nm;
                TN_HIP(hipEventRecord(pf.ev[set][di + 1], s));
            }
            ++di;
        }
        if (!err.empty()) break;
        const void* rp = node_ptr(p, d, ws, root, G.slice_base);
        const uint32_t* mk = mask_slot[gi] == (size_t)-1 ? nullptr : d_masks + mask_slot[gi] * d.mask_words;
        const uint64_t b0 = mk ? 0 : G.beta0;
        const uint64_t b1 = mk ? (1ull << p.batch_log2) : G.beta1;
        hipError_t e = launch_slice_sum(storage, rp, acc, p.root_log2, p.batch_log2, mk, b0, b1, s);
        if (e != hipSuccess) err = std::string("slice sum: ") + hipGetErrorString(e);
        if (pf.on && err.empty()) {
            if (pf.names[n_dep].empty()) pf.names[n_dep] = storage == ST_C128 ? "k_slice_sum<double2>" : "k_slice_sum<float2>";
            TN_HIP(hipEventRecord(pf.ev[set][n_dep + 1], s));
            pf.pending[set] = true;
        }
    }
    if (d_masks) {
        hipError_t e = hipFreeAsync(d_masks, s);
        if (err.empty() && e != hipSuccess) err = std::string("hipFreeAsync: ") + hipGetErrorString(e);
    }
    return err;
}

// ---------------------------------------------------------------- lanes

static void release_lane(Lane& ln);

uint64_t lane_stride(const Plan& p) { return (p.stats.workspace_bytes + 255) & ~uint64_t(255); }

uint64_t lanes_workspace_bytes(const Plan& p, int n) {
    return (uint64_t)std::max(0, n - 1) * lane_stride(p) + p.stats.workspace_bytes;
}

std::string set_lanes(DeviceState& d, int n) {
    if (n < 1 || n > kMaxLanes) return "lanes out of range (1.." + std::to_string(kMaxLanes) + ")";
    d.n_lanes = n;
    while ((int)d.lanes.size() > n - 1) {
        release_lane(*d.lanes.back());
        d.lanes.pop_back();
    }
    return "";
}

// One extra lane on the plan's device.
static std::string init_lane(Plan& p, const DeviceState& d, Lane& ln) {
    DeviceState& x = ln.d;
    x.device = d.device;
    x.plan_mem = d.plan_mem;
    x.plan_bytes = d.plan_bytes;
    x.mask_words = d.mask_words;
    x.prepared = true;
    if (d.d_max) TN_HIP(hipMalloc(&x.d_max, sizeof(float) * p.tree.n_nodes()));
    TN_HIP(hipMalloc(&x.d_state, sizeof(GroupState)));
    TN_HIP(hipMemset(x.d_state, 0, sizeof(GroupState)));
    TN_HIP(hipStreamCreateWithFlags(&ln.stream, hipStreamNonBlocking));
    TN_HIP(hipEventCreateWithFlags(&ln.join, hipEventDisableTiming));
    ln.acc_n = 1ull << p.root_log2;
    TN_HIP(hipMalloc(&ln.acc, 16 * ln.acc_n));
    return "";
}

// Lanes 1 .. n-1, made once; a lane that fails to initialise is released
// and not kept.
static std::string make_lanes(Plan& p, DeviceState& d, int n) {
    if (!d.fork) TN_HIP(hipEventCreateWithFlags(&d.fork, hipEventDisableTiming));
    while ((int)d.lanes.size() < n - 1) {
        auto ln = std::make_unique<Lane>();
        std::string err = init_lane(p, d, *ln);
        if (!err.empty()) {
            release_lane(*ln);
            return err;
        }
        d.lanes.push_back(std::move(ln));
    }
    return "";
}

std::string run_lanes(Plan& p, DeviceState& d, void* ws, size_t ws_bytes, double* acc,
                      const std::vector<Group>& groups, hipStream_t s) {
    int L = d.n_lanes;
    const uint64_t stride = lane_stride(p);
    if (ws_bytes < p.stats.workspace_bytes) return "workspace too small";
    L = (int)std::min<uint64_t>((uint64_t)L, 1 + (ws_bytes - p.stats.workspace_bytes) / stride);
    bool plain = !d.prof.on;
    for (const Group& g : groups) plain = plain && g.mask.empty();
    if (L < 2 || !plain || groups.size() < 2 * (size_t)L) return run_groups(p, d, ws, acc, groups, s);
    std::string err = make_lanes(p, d, L);
    if (!err.empty()) return err;
    const size_t n = groups.size();
    auto part = [&](int i) {
        return std::vector<Group>(groups.begin() + (n * i) / L, groups.begin() + (n * (i + 1)) / L);
    };
    TN_HIP(hipEventRecord(d.fork, s));
    for (int i = 1; i < L; ++i) {
        Lane& ln = *d.lanes[i - 1];
        TN_HIP(hipStreamWaitEvent(ln.stream, d.fork, 0));
        // the static max slots (leaves, slice-invariant tensors) as the plan has them now
        if (d.d_max && p.n_static_slots > 0)
            TN_HIP(hipMemcpyAsync(ln.d.d_max, d.d_max, sizeof(float) * p.n_static_slots, hipMemcpyDeviceToDevice,
                                  ln.stream));
        TN_HIP(launch_acc_zero(ln.acc, ln.acc_n, ln.stream));
    }
    err = run_groups(p, d, ws, acc, part(0), s);
    for (int i = 1; i < L && err.empty(); ++i) {
        Lane& ln = *d.lanes[i - 1];
        err = run_groups(p, ln.d, (unsigned char*)ws + (uint64_t)i * stride, ln.acc, part(i), ln.stream);
        if (err.empty()) {
            hipError_t e = hipEventRecord(ln.join, ln.stream);
            if (e != hipSuccess) err = std::string("hipEventRecord: ") + hipGetErrorString(e);
        }
    }
    if (!err.empty()) return err;
    for (int i = 1; i < L; ++i) {
        Lane& ln = *d.lanes[i - 1];
        TN_HIP(hipStreamWaitEvent(s, ln.join, 0));
        TN_HIP(launch_acc_add(acc, ln.acc, ln.acc_n, s));
    }
    return "";
}

// ------------------------------------------------------------- autotune

namespace {

struct Candidate {
    int kernel, tile, splitk;
};

// Every kernel configuration that can run a step of this shape.
std::vector<Candidate> candidates(const Step& st, tn_precision prec) {
    std::vector<Candidate> c;
    if (mfma_capable(prec) && st.m_log >= 4 && st.n_log >= 3 && st.k_log >= 1)
        for (int t = 0; t < kNumMfmaTiles; ++t)
            if (kMfmaTiles[t].tm_log <= st.m_log && kMfmaTiles[t].tn_log <= st.n_log) c.push_back({K_MFMA, t, 0});
    if (skinny_ok(st.m_log, st.n_log, st.k_log, st.b_log, prec)) c.push_back({K_SKINNY, 0, 0});
    for (int t = 0; t < kNumPanelTiles; ++t)
        if (panel_ok(st.m_log, st.n_log, st.k_log, st.b_log, prec, t)) {
            c.push_back({K_PANEL, t, 0});
            if (prec == TN_C64) {
                c.push_back({K_PANEL, t | 16, 0});        // non-temporal A loads
                c.push_back({K_PANEL, t | 32, 0});        // three real products per complex product
                c.push_back({K_PANEL, t | 32 | 16, 0});
                if (t & 1) c.push_back({K_PANEL, t | 32 | 128, 0});   // A staged in LDS by direct loads
            } else {
                c.push_back({K_PANEL, t | 4, 0});        // FP32 panel in a mixed form
                c.push_back({K_PANEL, t | 4 | 16, 0});
                c.push_back({K_PANEL, t | 4 | 32, 0});
                c.push_back({K_PANEL, t | 4 | 32 | 16, 0});
                c.push_back({K_PANEL, t | 8, 0});        // A split in registers, no separate pass
                c.push_back({K_PANEL, t | 8 | 16, 0});
            }
        }
    if (lp_prec(prec) && panel_ok(st.m_log, st.n_log, st.k_log, st.b_log, prec, 64 | 1)) {
        c.push_back({K_PANEL, 64 | 1, 0});   // 128 complex columns per block, KC = 16
        c.push_back({K_PANEL, 64 | 1 | 8, 0});
        c.push_back({K_PANEL, 64 | 1 | 8 | 16, 0});
    }
    c.push_back({K_SMALL, 0, 0});
    if (st.k_log <= 4 && st.n_log <= 4 && st.m_log >= (prec == TN_C128 ? 8 : 9) &&
        st.b_log <= 16)
        c.push_back({K_STREAM, 0, 0});
    if (st.kernel == K_SPLITK) c.push_back({K_SPLITK, 0, st.splitk_log});
    return c;
}

std::string shape_key(const std::string& arch, const Step& st, tn_precision prec) {
    return arch + " " + std::to_string(st.m_log) + " " + std::to_string(st.n_log) + " " + std::to_string(st.k_log) +
           " " + std::to_string(st.b_log) + " " + std::to_string((int)prec);
}

}  // namespace

std::string autotune(Plan& p, DeviceState& d, void* ws, double* acc, const char* cache_path, int reps, int& n_tuned,
                     hipStream_t s) {
    n_tuned = 0;
    reps = std::max(1, std::min(reps, 50));
    hipDeviceProp_t prop;
    int dev = 0;
    TN_HIP(hipGetDevice(&dev));
    TN_HIP(hipGetDeviceProperties(&prop, dev));
    std::string arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    std::map<std::string, std::pair<int, int>> cache;   // key -> (kernel, tile)
    if (cache_path) {
        FILE* f = std::fopen(cache_path, "r");
        if (f) {
            char a[64];
            int m, n, k, b, pr, ker, tile;
            while (std::fscanf(f, "%63s %d %d %d %d %d %d %d", a, &m, &n, &k, &b, &pr, &ker, &tile) == 8) {
                Step st{};
                st.m_log = m;
                st.n_log = n;
                st.k_log = k;
                st.b_log = b;
                cache[shape_key(a, st, (tn_precision)pr)] = {ker, tile};
            }
            std::fclose(f);
        }
    }
    // walk one real launch group step by step: each step is timed on the
    // operands its producers just wrote, then run with the chosen tile
    std::string err;
    if (d.d_max) TN_HIP(launch_fill(d.d_max + p.n_static_slots, (uint64_t)(p.tree.n_nodes() - p.n_static_slots), s));
    hipEvent_t e0, e1;
    TN_HIP(hipEventCreate(&e0));
    TN_HIP(hipEventCreate(&e1));
    std::map<std::string, std::pair<int, int>> decided;
    for (Step& st : p.steps) {
        if (st.invariant) continue;
        void* A = node_ptr(p, d, ws, st.a_node, 0);
        void* B = node_ptr(p, d, ws, st.b_node, 0);
        void* C = (unsigned char*)ws + st.c_off * (uint64_t)p.esize;
        const std::string key = shape_key(arch, st, p.opts.prec);
        const std::pair<int, int>* hit = nullptr;
        auto ci = cache.find(key);
        if (ci != cache.end()) hit = &ci->second;
        else {
            auto di = decided.find(key);
            if (di != decided.end()) hit = &di->second;
        }
        if (hit) {
            if (hit->first != K_SPLITK || st.kernel == K_SPLITK) {   // split-K needs planned scratch
                st.kernel = hit->first;
                st.tile = hit->second;
                if (st.kernel != K_SPLITK) st.splitk_log = 0;
            }
        } else {
            float best_ms = -1.f;
            Candidate best{st.kernel, st.tile, st.splitk_log};
            const Step orig = st;
            for (const Candidate& c : candidates(orig, p.opts.prec)) {
                st.kernel = c.kernel;
                st.tile = c.tile;
                st.splitk_log = c.kernel == K_SPLITK ? orig.splitk_log : 0;
                err = launch_step(p, d, st, A, B, C, ws, s);   // warm-up
                if (!err.empty()) break;
                std::vector<float> t;
                for (int r = 0; r < reps && err.empty(); ++r) {
                    TN_HIP(hipEventRecord(e0, s));
                    err = launch_step(p, d, st, A, B, C, ws, s);
                    TN_HIP(hipEventRecord(e1, s));
                    TN_HIP(hipEventSynchronize(e1));
                    float ms = 0.f;
                    TN_HIP(hipEventElapsedTime(&ms, e0, e1));
                    t.push_back(ms);
                }
                if (!err.empty()) break;
                std::sort(t.begin(), t.end());
                const float med = t[t.size() / 2];
                if (std::getenv("TN_TUNE_LOG"))
                    std::fprintf(stderr, "tune m%d n%d k%d b%d: kernel %d tile %d %.1f us\n", st.m_log, st.n_log,
                                 st.k_log, st.b_log, c.kernel, c.tile, 1e3 * med);
                if (best_ms < 0 || med < best_ms) {
                    best_ms = med;
                    best = c;
                }
            }
            st = orig;
            if (!err.empty()) break;
            st.kernel = best.kernel;
            st.tile = best.tile;
            st.splitk_log = best.kernel == K_SPLITK ? orig.splitk_log : 0;
            decided[key] = {best.kernel, best.tile};
            ++n_tuned;
        }
        err = launch_step(p, d, st, A, B, C, ws, s);   // the real output for the next steps
        if (!err.empty()) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!err.empty()) return err;
    // the captured graphs used the old choices
    err = drop_graphs(d);
    if (!err.empty()) return err;
    if (cache_path && !decided.empty()) {
        FILE* f = std::fopen(cache_path, "a");
        if (f) {
            for (auto& kv : decided) std::fprintf(f, "%s %d %d\n", kv.first.c_str(), kv.second.first, kv.second.second);
            std::fclose(f);
        }
    }
    return "";
}

std::vector<std::pair<int, int>> step_candidates(const Plan& p, int step) {
    std::vector<std::pair<int, int>> out;
    if (step < 0 || step >= (int)p.steps.size()) return out;
    for (const Candidate& c : candidates(p.steps[step], p.opts.prec)) out.push_back({c.kernel, c.tile});
    return out;
}

std::string set_step_kernel(Plan& p, DeviceState& d, int step, int kernel, int tile) {
    if (step < 0 || step >= (int)p.steps.size()) return "step out of range";
    Step& st = p.steps[step];
    bool ok = false;
    for (const Candidate& c : candidates(st, p.opts.prec)) ok |= c.kernel == kernel && c.tile == tile;
    if (!ok) return "not a candidate configuration of this step";
    if (kernel != K_SPLITK) st.splitk_log = 0;
    st.kernel = kernel;
    st.tile = tile;
    return drop_graphs(d);   // the captured graphs used the old choice
}

static void release_lane(Lane& ln) {
    if (ln.stream) (void)hipStreamSynchronize(ln.stream);
    ln.d.plan_mem = nullptr;   // the plan's, freed with the plan's state
    release(ln.d);
    if (ln.join) (void)hipEventDestroy(ln.join);
    if (ln.stream) (void)hipStreamDestroy(ln.stream);
    if (ln.acc) (void)hipFree(ln.acc);
    ln = Lane();
}

void release(DeviceState& d) {
    for (auto& ln : d.lanes) release_lane(*ln);
    d.lanes.clear();
    if (d.fork) (void)hipEventDestroy(d.fork);
    (void)drop_graphs(d);
    if (d.g_done) (void)hipEventDestroy(d.g_done);
    if (d.cap_stream) (void)hipStreamDestroy(d.cap_stream);
    if (d.d_state) (void)hipFree(d.d_state);
    for (int set = 0; set < 2; ++set)
        for (auto ev : d.prof.ev[set]) (void)hipEventDestroy(ev);
    if (d.plan_mem) (void)hipFree(d.plan_mem);
    if (d.d_mask) (void)hipFree(d.d_mask);
    if (d.d_part) (void)hipFree(d.d_part);
    if (d.d_max) (void)hipFree(d.d_max);
    d = DeviceState();
}

}  // namespace tn
