// extern "C" entry points declared in include/tn.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "exec.hpp"
#include "mix.hpp"
#include "sample.hpp"
#include "mlp.hpp"
#include "plan.hpp"

struct tn_plan_s {
    tn::Plan plan;
    tn::DeviceState dev;
    // big-head split: the tail plan (tail network + a leaf for v_head)
    tn_plan_s* tail = nullptr;
};

struct tn_mlp_s {
    tn::Mlp m;
    std::vector<float> fmin, fmax;
    float margin = 0.f;
    int device = -1;
};

namespace {

thread_local std::string g_err;

tn_status fail(tn_status s, const std::string& m) {
    g_err = m;
    return s;
}

tn_status from_err(const std::string& e) {
    if (e.empty()) return TN_OK;
    return fail(TN_EDEVICE, e);
}

}  // namespace

extern "C" {

const char* tn_last_error(void) { return g_err.c_str(); }

tn_status tn_plan(const tn_circuit* c, const int32_t* open_q, int32_t n_open, const int32_t* fixed_q,
                  const uint8_t* fixed_bits, int32_t n_fixed, const tn_tree* tree, const tn_edge* sliced,
                  int32_t n_sliced, const tn_plan_opts* opts, tn_plan_t* out) {
    if (!out) return fail(TN_EINVAL, "out is NULL");
    *out = nullptr;
    if (!c) return fail(TN_EINVAL, "circuit is NULL");
    if (n_open < 0 || n_fixed < 0 || (n_open > 0 && !open_q) || (n_fixed > 0 && (!fixed_q || !fixed_bits)))
        return fail(TN_EINVAL, "bad open/fixed qubit arrays");
    if (n_sliced > 0 && !sliced) return fail(TN_EINVAL, "sliced is NULL");
    if (tree && tree->n_steps > 0 && (!tree->lhs || !tree->rhs)) return fail(TN_EINVAL, "bad tree arrays");
    if (n_open > 40) return fail(TN_EUNSUPPORTED, "more than 40 open qubits");
    try {
        std::vector<int> o(open_q, open_q + n_open), f(fixed_q, fixed_q + n_fixed);
        std::vector<uint8_t> b(fixed_bits, fixed_bits + n_fixed);
        tn_plan_opts op = opts ? *opts : tn::default_opts();
        tn::CostModel cm;
        const tn::CostModel* cmp = nullptr;
        if (op.cost_model == 1 && op.model) {
            const tn_mlp_s* mm = op.model;
            if (mm->m.d_in != tn::kStepFeatures) return fail(TN_EINVAL, "model input width is not TN_STEP_FEATURES");
            cm.predict = [mm](const std::vector<float>& feats, int rows, std::vector<float>& out) -> std::string {
                // the model's own forward kernel, on its device
                tn::Mlp& net = const_cast<tn::Mlp&>(mm->m);
                float *dx = nullptr, *dy = nullptr;
                if (hipMalloc(&dx, sizeof(float) * feats.size()) != hipSuccess ||
                    hipMalloc(&dy, sizeof(float) * rows) != hipSuccess)
                    return "hipMalloc failed";
                std::string e;
                if (hipMemcpy(dx, feats.data(), sizeof(float) * feats.size(), hipMemcpyHostToDevice) != hipSuccess)
                    e = "upload failed";
                if (e.empty()) e = net.forward(dx, rows, dy, nullptr);
                out.assign(rows, 0.f);
                if (e.empty() && hipMemcpy(out.data(), dy, sizeof(float) * rows, hipMemcpyDeviceToHost) != hipSuccess)
                    e = "download failed";
                (void)hipFree(dx);
                (void)hipFree(dy);
                return e;
            };
            cm.in_support = [mm](const float* row) {
                if (mm->fmin.empty()) return true;
                for (size_t i = 0; i < mm->fmin.size(); ++i)
                    if (row[i] < mm->fmin[i] - mm->margin || row[i] > mm->fmax[i] + mm->margin) return false;
                return true;
            };
            cmp = &cm;
        }
        auto* h = new tn_plan_s;
        std::string err = tn::make_plan(*c, o, f, b, tree, sliced, n_sliced, op, h->plan, cmp);
        if (!err.empty()) {
            delete h;
            return fail(TN_EINVAL, err);
        }
        *out = h;
        return TN_OK;
    } catch (const std::bad_alloc&) {
        return fail(TN_ENOMEM, "host allocation failed");
    } catch (const std::exception& e) {
        return fail(TN_EINVAL, e.what());
    }
}

tn_status tn_plan_stats_get(tn_plan_t p, tn_plan_stats* out) {
    if (!p || !out) return fail(TN_EINVAL, "NULL argument");
    *out = p->plan.stats;
    out->graph_replays = p->dev.graph_replays;
    out->graph_launches = p->dev.graph_launches;
    for (const auto& ln : p->dev.lanes) {
        out->graph_replays += ln->d.graph_replays;
        out->graph_launches += ln->d.graph_launches;
    }
    out->lanes = p->dev.n_lanes;
    out->lanes_workspace_bytes = tn::lanes_workspace_bytes(p->plan, p->dev.n_lanes);
    return TN_OK;
}

tn_status tn_plan_sliced_edges(tn_plan_t p, tn_edge* out, int32_t cap, int32_t* n) {
    if (!p || !n || (cap > 0 && !out)) return fail(TN_EINVAL, "NULL argument");
    const auto& s = p->plan.sliced;
    *n = (int32_t)s.size();
    for (int32_t i = 0; i < cap && i < (int32_t)s.size(); ++i) {
        out[i].qubit = p->plan.net.edge_name[s[i]].q;
        out[i].segment = p->plan.net.edge_name[s[i]].t;
    }
    return TN_OK;
}

tn_status tn_plan_export_json(tn_plan_t p, char* buf, size_t cap, size_t* need) {
    if (!p || !need) return fail(TN_EINVAL, "NULL argument");
    try {
        std::string j = tn::plan_to_json(p->plan);
        *need = j.size() + 1;
        if (buf && cap > 0) {
            size_t n = std::min(cap - 1, j.size());
            std::memcpy(buf, j.data(), n);
            buf[n] = 0;
        }
        return TN_OK;
    } catch (const std::bad_alloc&) {
        return fail(TN_ENOMEM, "host allocation failed");
    }
}

static tn_status contract_groups(tn_plan_t p, void* ws, size_t ws_bytes, double* acc,
                                 const std::vector<tn::Group>& groups, void* stream) {
    if (!ws || !acc) return fail(TN_EINVAL, "NULL device buffer");
    if (ws_bytes < p->plan.stats.workspace_bytes)
        return fail(TN_EINVAL, "workspace too small: need " + std::to_string(p->plan.stats.workspace_bytes));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    try {
        std::string e = tn::prepare(p->plan, p->dev, s);
        if (!e.empty()) return fail(TN_EDEVICE, e);
        return from_err(tn::run_lanes(p->plan, p->dev, ws, ws_bytes, acc, groups, s));
    } catch (const std::bad_alloc&) {
        return fail(TN_ENOMEM, "host allocation failed");
    }
}

tn_status tn_contract_slices(tn_plan_t p, void* d_workspace, size_t ws_bytes, double* d_acc, uint64_t slice_begin,
                             uint64_t slice_end, void* hip_stream) {
    if (!p) return fail(TN_EINVAL, "plan is NULL");
    const uint64_t n = p->plan.stats.n_slices;
    if (slice_begin > slice_end || slice_end > n) return fail(TN_EINVAL, "slice range out of bounds");
    if (slice_begin == slice_end) return TN_OK;
    const int b = p->plan.batch_log2;
    const uint64_t B = 1ull << b;
    std::vector<tn::Group> groups;
    for (uint64_t o = slice_begin >> b; o <= (slice_end - 1) >> b; ++o) {
        tn::Group g;
        g.slice_base = o << b;
        g.beta0 = (o == (slice_begin >> b)) ? (slice_begin & (B - 1)) : 0;
        g.beta1 = (o == ((slice_end - 1) >> b)) ? ((slice_end - 1) & (B - 1)) + 1 : B;
        groups.push_back(g);
    }
    return contract_groups(p, d_workspace, ws_bytes, d_acc, groups, hip_stream);
}

tn_status tn_contract_slice_list(tn_plan_t p, void* d_workspace, size_t ws_bytes, double* d_acc,
                                 const uint64_t* h_slice_ids, uint64_t n_ids, void* hip_stream) {
    if (!p) return fail(TN_EINVAL, "plan is NULL");
    if (n_ids == 0) return TN_OK;
    if (!h_slice_ids) return fail(TN_EINVAL, "slice id list is NULL");
    const uint64_t n = p->plan.stats.n_slices;
    const int b = p->plan.batch_log2;
    const uint64_t B = 1ull << b;
    std::vector<uint64_t> ids(h_slice_ids, h_slice_ids + n_ids);
    std::sort(ids.begin(), ids.end());
    for (size_t i = 0; i < ids.size(); ++i) {
        if (ids[i] >= n) return fail(TN_EINVAL, "slice id out of range");
        if (i && ids[i] == ids[i - 1]) return fail(TN_EINVAL, "slice id repeated");
    }
    std::vector<tn::Group> groups;
    const size_t words = std::max<size_t>(1, (B + 31) / 32);
    for (size_t i = 0; i < ids.size();) {
        const uint64_t o = ids[i] >> b;
        tn::Group g;
        g.slice_base = o << b;
        g.mask.assign(words, 0);
        size_t cnt = 0;
        while (i < ids.size() && (ids[i] >> b) == o) {
            const uint64_t be = ids[i] & (B - 1);
            g.mask[be >> 5] |= 1u << (be & 31);
            ++i;
            ++cnt;
        }
        if (cnt == B) {   // full group: plain range
            g.mask.clear();
            g.beta0 = 0;
            g.beta1 = B;
        }
        groups.push_back(std::move(g));
    }
    return contract_groups(p, d_workspace, ws_bytes, d_acc, groups, hip_stream);
}

tn_status tn_amplitudes(tn_plan_t p, const double* d_acc, double* d_amps, void* d_workspace, size_t ws_bytes,
                        void* hip_stream) {
    if (!p || !d_acc || !d_amps) return fail(TN_EINVAL, "NULL argument");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    if (p->plan.tail) {
        // big-head: v_head (the accumulator, summed over slices) becomes the
        // last leaf of the tail network, which is contracted once in
        // complex128 into A[s2] = sum_c T_tail[s2, c] v_head[c]
        const int n_c = p->plan.stats.n_c, n_open = p->plan.stats.n_open;
        if (!d_workspace || ws_bytes < p->plan.stats.tail_workspace_bytes)
            return fail(TN_EINVAL, "workspace smaller than stats.tail_workspace_bytes");
        try {
            if (!p->tail) {
                p->tail = new tn_plan_s;
                p->tail->plan = *p->plan.tail;
            }
            tn::Plan& tp = p->tail->plan;
            std::string err = tn::prepare(tp, p->tail->dev, s);   // tail-only steps, once
            if (!err.empty()) return fail(TN_EDEVICE, err);
            // interleaved float64 (re, im) has the layout of std::complex<double>
            std::vector<tn::cd> v(size_t(1) << n_c);
            hipError_t e = hipMemcpyAsync(v.data(), d_acc, sizeof(tn::cd) * v.size(), hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) return fail(TN_EDEVICE, std::string("v_head download: ") + hipGetErrorString(e));
            err = tn::upload_leaf(tp, p->tail->dev, tp.tree.n_leaves - 1, std::move(v), s);
            if (!err.empty()) return fail(TN_EDEVICE, err);
            if ((e = hipMemsetAsync(d_amps, 0, sizeof(double) * (2ull << n_open), s)) != hipSuccess)
                return fail(TN_EDEVICE, std::string("amplitudes: ") + hipGetErrorString(e));
            tn::Group g;
            g.slice_base = 0;
            g.beta0 = 0;
            g.beta1 = 1;
            return from_err(tn::run_groups(tp, p->tail->dev, d_workspace, d_amps, {g}, s));
        } catch (const std::bad_alloc&) {
            return fail(TN_ENOMEM, "host allocation failed");
        }
    }
    const uint64_t n = 2ull << p->plan.root_log2;
    hipError_t e = tn::launch_copy_acc(d_acc, d_amps, n, s);
    if (e != hipSuccess) return fail(TN_EDEVICE, std::string("copy: ") + hipGetErrorString(e));
    return TN_OK;
}

size_t tn_sample_workspace_bytes(int32_t n_open) {
    if (n_open < 0 || n_open > 34) return 0;
    return sizeof(double) * tn::sample_workspace_elems(1ull << n_open);
}

tn_status tn_sample(const double* d_amps, int32_t n_open, const double* d_uniform, uint64_t n_samples,
                    uint64_t* d_out, void* d_workspace, size_t ws_bytes, void* hip_stream) {
    if (!d_amps || !d_workspace || (n_samples > 0 && (!d_uniform || !d_out))) return fail(TN_EINVAL, "NULL argument");
    if (n_open < 0 || n_open > 34) return fail(TN_EINVAL, "n_open out of range");
    if (ws_bytes < tn_sample_workspace_bytes(n_open)) return fail(TN_EINVAL, "workspace smaller than tn_sample_workspace_bytes");
    hipError_t e = tn::launch_sample(d_amps, 1ull << n_open, d_uniform, n_samples, d_out,
                                     static_cast<double*>(d_workspace), reinterpret_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(TN_EDEVICE, std::string("sample: ") + hipGetErrorString(e));
    return TN_OK;
}

tn_status tn_sample_noalloc(const double* d_amps, int32_t n_open, const double* d_uniform, uint64_t n_samples,
                            uint64_t* d_out, void* hip_stream) {
    if (!d_amps || (n_samples > 0 && (!d_uniform || !d_out))) return fail(TN_EINVAL, "NULL argument");
    if (n_open < 0 || n_open > tn::kStaticSampleMaxOpen)
        return fail(TN_EINVAL, "n_open above the allocation-free limit of " +
                                   std::to_string(tn::kStaticSampleMaxOpen));
    hipError_t e = tn::launch_sample_static(d_amps, 1ull << n_open, d_uniform, n_samples, d_out,
                                            reinterpret_cast<hipStream_t>(hip_stream));
    if (e != hipSuccess) return fail(TN_EDEVICE, std::string("sample: ") + hipGetErrorString(e));
    return TN_OK;
}

size_t tn_mix_workspace_bytes(int32_t n_open) {
    if (n_open < 0 || n_open > 34) return 0;
    return tn::mix_workspace_bytes(1ull << n_open);
}

tn_status tn_mix_topk(const double* d_amps, int32_t n_qubits, const int32_t* open_q, int32_t n_open,
                      const int32_t* fixed_q, const uint8_t* fixed_bits, int32_t n_fixed, uint64_t k,
                      const uint64_t* d_random_words, uint64_t n_random, uint64_t* d_out, void* d_workspace,
                      size_t ws_bytes, tn_mix_result* out, void* hip_stream) {
    if (!d_amps || !out || (n_open > 0 && !open_q) || (n_fixed > 0 && (!fixed_q || !fixed_bits)))
        return fail(TN_EINVAL, "NULL argument");
    if (n_open < 0 || n_open > 34 || n_fixed < 0 || n_qubits != n_open + n_fixed || n_qubits > 64)
        return fail(TN_EINVAL, "bad sizes (n_qubits = n_open + n_fixed <= 64, n_open <= 34)");
    const uint64_t L = 1ull << n_open;
    if (k > L) return fail(TN_EINVAL, "k exceeds the number of computed amplitudes");
    if ((k + n_random > 0 && !d_out) || (n_random > 0 && !d_random_words)) return fail(TN_EINVAL, "NULL buffer");
    if (!d_workspace || ws_bytes < tn_mix_workspace_bytes(n_open))
        return fail(TN_EINVAL, "workspace smaller than tn_mix_workspace_bytes");
    tn::MixBits mb{};
    std::vector<char> seen(n_qubits, 0);
    for (int i = 0; i < n_open + n_fixed; ++i) {
        const int q = i < n_open ? open_q[i] : fixed_q[i - n_open];
        if (q < 0 || q >= n_qubits || seen[q]) return fail(TN_EINVAL, "open and fixed qubits must partition 0..n-1");
        seen[q] = 1;
    }
    for (int j = 0; j < n_open; ++j) {
        if (j && open_q[j] <= open_q[j - 1]) return fail(TN_EINVAL, "open qubits must be ascending");
        mb.pos[j] = (uint8_t)(n_qubits - 1 - open_q[j]);
    }
    mb.n_open = n_open;
    for (int i = 0; i < n_fixed; ++i)
        if (fixed_bits[i]) mb.base |= 1ull << (n_qubits - 1 - fixed_q[i]);
    double p_top = 0.0;
    std::string err = tn::mix_topk(d_amps, L, k, mb, d_random_words, n_random, n_qubits, d_out, d_workspace,
                                   reinterpret_cast<hipStream_t>(hip_stream), p_top);
    if (!err.empty()) return fail(TN_EDEVICE, err);
    const double two_n = std::ldexp(1.0, n_qubits);
    out->P_top = p_top;
    out->F_top = k ? two_n / (double)k * p_top - 1.0 : 0.0;
    const double n_all = (double)k + (double)n_random;
    out->F_mix_expected = n_all > 0 ? (two_n * p_top + (double)n_random) / n_all - 1.0 : 0.0;
    return TN_OK;
}

tn_status tn_xeb(const double* d_amps, int32_t n_open, int32_t n_qubits, double weight, const int64_t* ks,
                 int32_t n_ks, double* h_topk, tn_xeb_result* out, void* hip_stream) {
    if (!d_amps || !out) return fail(TN_EINVAL, "NULL argument");
    // 2^n_qubits must be a finite double (Eq. (1) scales by it)
    if (n_open < 0 || n_open > 40 || n_qubits < n_open || n_qubits > 1023) return fail(TN_EINVAL, "bad sizes");
    if (n_ks < 0 || (n_ks > 0 && (!ks || !h_topk))) return fail(TN_EINVAL, "bad top-k arrays");
    if (!(weight > 0)) return fail(TN_EINVAL, "weight must be positive");
    const uint64_t L = 1ull << n_open;
    for (int i = 0; i < n_ks; ++i)
        if (ks[i] < 1 || (uint64_t)ks[i] > L) return fail(TN_EINVAL, "top-k size out of range");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    const int blocks = (int)std::min<uint64_t>(1024, (L + 255) / 256);
    double* part = nullptr;
    hipError_t e = hipMallocAsync((void**)&part, sizeof(double) * 5 * blocks, s);
    if (e != hipSuccess) return fail(TN_EDEVICE, std::string("hipMallocAsync: ") + hipGetErrorString(e));
    std::vector<double> h(5 * blocks);
    auto done = [&](tn_status st) {
        (void)hipFreeAsync(part, s);
        (void)hipStreamSynchronize(s);
        return st;
    };
    if ((e = tn::launch_xeb_partials(d_amps, L, weight, part, blocks, s)) != hipSuccess ||
        (e = hipMemcpyAsync(h.data(), part, sizeof(double) * 4 * blocks, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return done(fail(TN_EDEVICE, std::string("xeb: ") + hipGetErrorString(e)));
    double s1 = 0, s2 = 0, mx = 0, mn = 1e300;
    for (int b = 0; b < blocks; ++b) {
        s1 += h[4 * b];
        s2 += h[4 * b + 1];
        mx = std::max(mx, h[4 * b + 2]);
        mn = std::min(mn, h[4 * b + 3]);
    }
    if ((e = tn::launch_xeb_cond(d_amps, L, weight, s1 > 0 ? 1.0 / s1 : 0.0, part + 4 * blocks, blocks, s)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(h.data() + 4 * blocks, part + 4 * blocks, sizeof(double) * blocks, hipMemcpyDeviceToHost,
                            s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return done(fail(TN_EDEVICE, std::string("xeb: ") + hipGetErrorString(e)));
    double cs = 0;
    for (int b = 0; b < blocks; ++b) cs += h[4 * blocks + b];
    const double two_n = std::ldexp(1.0, n_qubits);
    out->P_s1 = s1;
    out->F_unif = two_n / (double)L * s1 - 1.0;
    out->F_self = s1 > 0 ? two_n * s2 / s1 - 1.0 : -1.0;
    out->cond_xeb = cs - 1.0;   // 2^n2 / L * sum P(s2|s1) - 1 with L = 2^n2
    out->p_max = mx;
    out->p_min = mn;
    if (n_ks > 0) {
        std::vector<double> a(2 * L);
        if ((e = hipMemcpyAsync(a.data(), d_amps, sizeof(double) * 2 * L, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return done(fail(TN_EDEVICE, std::string("xeb copy: ") + hipGetErrorString(e)));
        std::vector<double> pr(L);
        for (uint64_t i = 0; i < L; ++i) pr[i] = weight * (a[2 * i] * a[2 * i] + a[2 * i + 1] * a[2 * i + 1]);
        std::sort(pr.begin(), pr.end(), [](double x, double y) { return x > y; });
        std::vector<int64_t> order(n_ks);
        for (int i = 0; i < n_ks; ++i) order[i] = i;
        std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return ks[x] < ks[y]; });
        double c = 0;
        uint64_t pos = 0;
        for (int64_t oi : order) {
            while (pos < (uint64_t)ks[oi]) c += pr[pos++];
            h_topk[oi] = two_n / (double)ks[oi] * c - 1.0;
        }
    }
    return done(TN_OK);
}

tn_status tn_plan_set_lanes(tn_plan_t p, int32_t lanes) {
    if (!p) return fail(TN_EINVAL, "plan is NULL");
    if (lanes < 1 || lanes > tn::kMaxLanes) return fail(TN_EINVAL, "lanes out of range");
    try {
        return from_err(tn::set_lanes(p->dev, lanes));
    } catch (const std::bad_alloc&) {
        return fail(TN_ENOMEM, "host allocation failed");
    }
}

tn_status tn_plan_set_profiling(tn_plan_t p, int32_t enable) {
    if (!p) return fail(TN_EINVAL, "plan is NULL");
    return from_err(tn::profile_enable(p->plan, p->dev, enable != 0));
}

tn_status tn_plan_step_profile(tn_plan_t p, tn_step_profile* out, int32_t cap, int32_t* n) {
    if (!p || !n || (cap > 0 && !out)) return fail(TN_EINVAL, "NULL argument");
    tn::Profiler& pf = p->dev.prof;
    std::string e = tn::profile_harvest(p->dev);
    if (!e.empty()) return fail(TN_EDEVICE, e);
    *n = (int32_t)pf.ms.size();
    int di = 0;
    for (const tn::Step& st : p->plan.steps) {
        if (st.invariant) continue;
        if (di < cap) {
            tn_step_profile& o = out[di];
            std::memset(&o, 0, sizeof(o));
            o.m_log = st.m_log;
            o.n_log = st.n_log;
            o.k_log = st.k_log;
            o.b_log = st.b_log;
            o.kernel = st.kernel;
            o.tile = st.tile;
            o.cmacs = st.cmacs;
            o.bytes = st.bytes;
            o.total_ms = di < (int)pf.ms.size() ? pf.ms[di] : 0.0;
            o.launches = di < (int)pf.launches.size() ? pf.launches[di] : 0;
            if (di < (int)pf.names.size()) std::strncpy(o.kernel_name, pf.names[di].c_str(), sizeof(o.kernel_name) - 1);
        }
        ++di;
    }
    if (di < cap && di < (int)pf.ms.size()) {   // slice sum
        tn_step_profile& o = out[di];
        std::memset(&o, 0, sizeof(o));
        o.m_log = p->plan.root_log2;
        o.b_log = p->plan.batch_log2;
        o.kernel = -1;
        o.cmacs = 0;
        o.bytes = (double)p->plan.esize * std::ldexp(1.0, p->plan.root_log2 + p->plan.batch_log2) +
                  32.0 * std::ldexp(1.0, p->plan.root_log2);
        o.total_ms = pf.ms[di];
        o.launches = pf.launches[di];
        std::strncpy(o.kernel_name, pf.names[di].c_str(), sizeof(o.kernel_name) - 1);
    }
    return TN_OK;
}

tn_status tn_plan_autotune(tn_plan_t p, void* d_workspace, size_t ws_bytes, double* d_acc_scratch,
                           const char* cache_path, int32_t reps, int32_t* n_tuned, void* hip_stream) {
    if (!p || !d_workspace || !d_acc_scratch || !n_tuned) return fail(TN_EINVAL, "NULL argument");
    if (ws_bytes < p->plan.stats.workspace_bytes) return fail(TN_EINVAL, "workspace too small");
    if (p->dev.prof.on) return fail(TN_ESTATE, "disable step timing before autotuning");
    hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
    try {
        std::string e = tn::prepare(p->plan, p->dev, s);
        if (!e.empty()) return fail(TN_EDEVICE, e);
        int nt = 0;
        e = tn::autotune(p->plan, p->dev, d_workspace, d_acc_scratch, cache_path, reps, nt, s);
        *n_tuned = nt;
        if (!e.empty()) return fail(TN_EDEVICE, e);
        // kernel counts in the stats follow the new choices
        p->plan.stats.n_dense_steps = p->plan.stats.n_small_steps = 0;
        for (const tn::Step& st : p->plan.steps)
            (st.kernel == tn::K_MFMA || st.kernel == tn::K_SKINNY || st.kernel == tn::K_PANEL ? p->plan.stats.n_dense_steps : p->plan.stats.n_small_steps)++;
        return TN_OK;
    } catch (const std::bad_alloc&) {
        return fail(TN_ENOMEM, "host allocation failed");
    }
}

tn_status tn_choose_open_qubits(const tn_circuit* c, int32_t n_open, const tn_plan_opts* opts, int32_t* h_open,
                                int32_t* n_cut) {
    if (!c || !h_open || !n_cut) return fail(TN_EINVAL, "NULL argument");
    try {
        std::vector<int> open;
        int cut = 0;
        const std::string e =
            tn::choose_open_qubits(*c, n_open, opts ? *opts : tn::default_opts(), open, cut);
        if (!e.empty()) return fail(TN_EINVAL, e);
        for (size_t i = 0; i < open.size(); ++i) h_open[i] = open[i];
        *n_cut = cut;
        return TN_OK;
    } catch (const std::bad_alloc&) {
        return fail(TN_ENOMEM, "host allocation failed");
    }
}

tn_status tn_plan_step_candidates(tn_plan_t p, int32_t step, int32_t* h_kernels, int32_t* h_tiles, int32_t cap,
                                  int32_t* n) {
    if (!p || !n || (cap > 0 && (!h_kernels || !h_tiles))) return fail(TN_EINVAL, "NULL argument");
    if (step < 0 || step >= (int)p->plan.steps.size()) return fail(TN_EINVAL, "step out of range");
    try {
        const auto c = tn::step_candidates(p->plan, step);
        *n = (int32_t)c.size();
        for (int32_t i = 0; i < cap && i < (int32_t)c.size(); ++i) {
            h_kernels[i] = c[i].first;
            h_tiles[i] = c[i].second;
        }
        return TN_OK;
    } catch (const std::bad_alloc&) {
        return fail(TN_ENOMEM, "host allocation failed");
    }
}

tn_status tn_plan_set_step_kernel(tn_plan_t p, int32_t step, int32_t kernel, int32_t tile) {
    if (!p) return fail(TN_EINVAL, "NULL argument");
    if (p->dev.prof.on) return fail(TN_ESTATE, "disable step timing before changing kernels");
    try {
        const std::string e = tn::set_step_kernel(p->plan, p->dev, step, kernel, tile);
        if (!e.empty()) return fail(TN_EINVAL, e);
        return TN_OK;
    } catch (const std::bad_alloc&) {
        return fail(TN_ENOMEM, "host allocation failed");
    }
}

tn_status tn_step_features(int32_t m_log, int32_t n_log, int32_t k_log, int32_t b_log, int32_t kernel,
                           tn_precision prec, float* out) {
    if (!out) return fail(TN_EINVAL, "NULL argument");
    tn::step_features(m_log, n_log, k_log, b_log, kernel, prec == TN_C128 ? 16 : 8, out);
    return TN_OK;
}

tn_status tn_plan_step_features(tn_plan_t p, float* h_out, int32_t cap_steps, int32_t* n_steps) {
    if (!p || !n_steps || (cap_steps > 0 && !h_out)) return fail(TN_EINVAL, "NULL argument");
    int i = 0;
    for (const tn::Step& st : p->plan.steps) {
        if (st.invariant) continue;
        if (i < cap_steps)
            tn::step_features(st.m_log, st.n_log, st.k_log, st.b_log, st.kernel, p->plan.esize,
                              h_out + (size_t)i * tn::kStepFeatures);
        ++i;
    }
    *n_steps = i;
    return TN_OK;
}

tn_status tn_mlp_create(int32_t d_in, int32_t hidden, uint64_t seed, tn_mlp_t* out) {
    if (!out || d_in < 1 || hidden < 1 || d_in > 4096 || hidden > 4096) return fail(TN_EINVAL, "bad arguments");
    *out = nullptr;
    try {
        auto* h = new tn_mlp_s;
        std::string e = h->m.create(d_in, hidden, seed);
        if (!e.empty()) {
            h->m.release();
            delete h;
            return fail(TN_EDEVICE, e);
        }
        (void)hipGetDevice(&h->device);
        *out = h;
        return TN_OK;
    } catch (const std::bad_alloc&) {
        return fail(TN_ENOMEM, "host allocation failed");
    }
}

tn_status tn_mlp_num_params(tn_mlp_t m, int64_t* n) {
    if (!m || !n) return fail(TN_EINVAL, "NULL argument");
    *n = m->m.n_params();
    return TN_OK;
}

tn_status tn_mlp_get_params(tn_mlp_t m, float* h, int64_t n) {
    if (!m || !h || n != m->m.n_params()) return fail(TN_EINVAL, "bad arguments");
    if (hipMemcpy(h, m->m.params, sizeof(float) * n, hipMemcpyDeviceToHost) != hipSuccess)
        return fail(TN_EDEVICE, "download failed");
    return TN_OK;
}

tn_status tn_mlp_set_params(tn_mlp_t m, const float* h, int64_t n) {
    if (!m || !h || n != m->m.n_params()) return fail(TN_EINVAL, "bad arguments");
    if (hipMemcpy(m->m.params, h, sizeof(float) * n, hipMemcpyHostToDevice) != hipSuccess)
        return fail(TN_EDEVICE, "upload failed");
    return TN_OK;
}

tn_status tn_mlp_forward(tn_mlp_t m, const float* d_x, int32_t batch, float* d_y, void* stream) {
    if (!m || !d_x || !d_y || batch < 1) return fail(TN_EINVAL, "bad arguments");
    return from_err(m->m.forward(d_x, batch, d_y, reinterpret_cast<hipStream_t>(stream)));
}

tn_status tn_mlp_gradient(tn_mlp_t m, const float* d_x, const float* d_t, int32_t batch, float* h_grads,
                          float* h_loss, void* stream) {
    if (!m || !d_x || !d_t || batch < 1) return fail(TN_EINVAL, "bad arguments");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    float loss = 0.f;
    std::string e = m->m.gradient(d_x, d_t, batch, &loss, s);
    if (!e.empty()) return fail(TN_EDEVICE, e);
    if (h_loss) *h_loss = loss;
    if (h_grads) {
        if (hipMemcpyAsync(h_grads, m->m.grads, sizeof(float) * m->m.n_params(), hipMemcpyDeviceToHost, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(TN_EDEVICE, "download failed");
    }
    return TN_OK;
}

tn_status tn_mlp_train_step(tn_mlp_t m, const float* d_x, const float* d_t, int32_t batch, float lr, float* h_loss,
                            void* stream) {
    if (!m || !d_x || !d_t || batch < 1 || !(lr > 0)) return fail(TN_EINVAL, "bad arguments");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    float loss = 0.f;
    std::string e = m->m.gradient(d_x, d_t, batch, h_loss ? &loss : nullptr, s);
    if (e.empty()) e = m->m.adam(lr, s);
    if (!e.empty()) return fail(TN_EDEVICE, e);
    if (h_loss) *h_loss = loss;
    return TN_OK;
}

tn_status tn_mlp_set_support(tn_mlp_t m, const float* h_min, const float* h_max, int32_t n_feat, float margin) {
    if (!m || !h_min || !h_max || n_feat != m->m.d_in) return fail(TN_EINVAL, "bad arguments");
    m->fmin.assign(h_min, h_min + n_feat);
    m->fmax.assign(h_max, h_max + n_feat);
    m->margin = margin;
    return TN_OK;
}

void tn_mlp_destroy(tn_mlp_t m) {
    if (!m) return;
    m->m.release();
    delete m;
}

void tn_plan_destroy(tn_plan_t p) {
    if (!p) return;
    if (p->tail) tn_plan_destroy(p->tail);
    if (p->dev.prepared || p->dev.plan_mem) {
        int cur = 0;
        if (hipGetDevice(&cur) == hipSuccess && p->dev.device >= 0 && cur != p->dev.device) {
            (void)hipSetDevice(p->dev.device);
            tn::release(p->dev);
            (void)hipSetDevice(cur);
        } else {
            tn::release(p->dev);
        }
    }
    delete p;
}

}  // extern "C"
