// Executor: uploads a plan's leaves, computes its slice-invariant subtrees
// once, then runs the slice-dependent steps of each launch group (2^b slices
// whose batch legs are contracted together) followed by the float64 slice
// sum ("summation of the final tensors", appendix B).
#include "exec.hpp"

#include <algorithm>
#include <cstring>

#include "tiles.hpp"

namespace tn {

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

std::string launch_step(const Plan& p, const Step& st, const void* A, const void* B, void* C, void* ws,
                        hipStream_t s) {
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    g.A = A;
    g.B = B;
    g.C = C;
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
    } else {
        const int m = st.m_log, n = st.n_log;
        g.split_log = st.kernel == K_SPLITK ? st.splitk_log : 0;
        const int k = st.k_log - g.split_log;
        const int r_log = (m + n >= 10) ? 2 : (m + n >= 9 ? 1 : 0);
        const int tile_log = std::min(8 + r_log, m + n);
        g.tm = std::min(m, tile_log);
        g.tn = std::min(n, tile_log - g.tm);
        R = 1 << std::max(0, g.tm + g.tn - 8);
        const int limit = (int)(32768 / esz);
        int tk = 0;
        while (tk < k && (2 << tk) * ((1 << g.tm) + (1 << g.tn)) <= limit) ++tk;
        g.tk = tk;
        if (g.split_log > 0) g.scratch = (unsigned char*)ws + st.scratch_off * (uint64_t)p.esize;
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
    hipError_t e;
    if (st.kernel == K_MFMA) {
        e = launch_mfma(0, st.tile, g, s);
    } else {
        e = launch_valu(storage, g, R, s);
        if (e == hipSuccess && g.split_log > 0) e = launch_splitk_reduce(storage, g, s);
    }
    if (e != hipSuccess) return std::string("step launch: ") + hipGetErrorString(e);
    return "";
}

}  // namespace

int storage_of(tn_precision p) {
    switch (p) {
        case TN_C128: return ST_C128;
        case TN_BF16: return ST_BF16;
        default: return ST_C64;
    }
}

std::string prepare(Plan& p, DeviceState& d, hipStream_t s) {
    int dev = 0;
    TN_HIP(hipGetDevice(&dev));
    if (d.prepared && d.device == dev) return "";
    if (d.prepared && d.device != dev) return "plan was prepared on another device";
    const int storage = storage_of(p.opts.prec);
    if (storage == ST_BF16) return "bf16 storage is not available in this build";
    d.device = dev;
    d.plan_bytes = std::max<uint64_t>(p.plan_elems, 64) * (uint64_t)p.esize;
    TN_HIP(hipMalloc(&d.plan_mem, d.plan_bytes));
    std::vector<unsigned char> host(d.plan_bytes, 0);
    for (int i = 0; i < p.tree.n_leaves; ++i)
        put_leaf(p.net.leaves[i], p.nodes[i].layout, storage, host.data() + p.nodes[i].off * p.esize);
    TN_HIP(hipMemcpy(d.plan_mem, host.data(), d.plan_bytes, hipMemcpyHostToDevice));
    for (const Step& st : p.steps) {
        if (!st.invariant) continue;
        void* A = node_ptr(p, d, nullptr, st.a_node, 0);
        void* B = node_ptr(p, d, nullptr, st.b_node, 0);
        void* C = (unsigned char*)d.plan_mem + st.c_off * (uint64_t)p.esize;
        if (st.kernel == K_SPLITK) return "split-K step in the slice-invariant part needs a workspace";
        std::string err = launch_step(p, st, A, B, C, nullptr, s);
        if (!err.empty()) return err;
    }
    d.mask_words = std::max<size_t>(1, ((size_t(1) << p.batch_log2) + 31) / 32);
    TN_HIP(hipStreamSynchronize(s));
    d.prepared = true;
    return "";
}

std::string run_groups(Plan& p, DeviceState& d, void* ws, double* acc, const std::vector<Group>& groups,
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
    for (size_t gi = 0; gi < groups.size() && err.empty(); ++gi) {
        const Group& G = groups[gi];
        for (const Step& st : p.steps) {
            if (st.invariant) continue;
            void* A = node_ptr(p, d, ws, st.a_node, G.slice_base);
            void* B = node_ptr(p, d, ws, st.b_node, G.slice_base);
            void* C = (unsigned char*)ws + st.c_off * (uint64_t)p.esize;
            err = launch_step(p, st, A, B, C, ws, s);
            if (!err.empty()) break;
        }
        if (!err.empty()) break;
        const void* rp = node_ptr(p, d, ws, root, G.slice_base);
        const uint32_t* mk = mask_slot[gi] == (size_t)-1 ? nullptr : d_masks + mask_slot[gi] * d.mask_words;
        const uint64_t b0 = mk ? 0 : G.beta0;
        const uint64_t b1 = mk ? (1ull << p.batch_log2) : G.beta1;
        hipError_t e = launch_slice_sum(storage, rp, acc, p.root_log2, p.batch_log2, mk, b0, b1, s);
        if (e != hipSuccess) err = std::string("slice sum: ") + hipGetErrorString(e);
    }
    if (d_masks) {
        hipError_t e = hipFreeAsync(d_masks, s);
        if (err.empty() && e != hipSuccess) err = std::string("hipFreeAsync: ") + hipGetErrorString(e);
    }
    return err;
}

void release(DeviceState& d) {
    if (d.plan_mem) (void)hipFree(d.plan_mem);
    if (d.d_mask) (void)hipFree(d.d_mask);
    if (d.d_part) (void)hipFree(d.d_part);
    d = DeviceState();
}

}  // namespace tn
