// Executor: runs a plan's steps on one HIP stream.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "kernels.hpp"
#include "plan.hpp"

namespace tn {

struct Profiler {
    bool on = false;
    std::vector<hipEvent_t> ev[2];      // per group parity: one event before each step + one at the end
    bool pending[2] = {false, false};
    std::vector<double> ms;             // per dependent step (+ slice sum)
    std::vector<uint64_t> launches;
    std::vector<std::string> names;
};

struct Lane;

struct DeviceState {
    int device = -1;
    void* plan_mem = nullptr;     // leaves + slice-invariant tensors
    size_t plan_bytes = 0;
    bool prepared = false;
    uint32_t* d_mask = nullptr;   // batch-slot masks for slice lists
    size_t mask_words = 0;
    double* d_part = nullptr;     // XEB partials
    float* d_max = nullptr;       // per-tensor max |re|,|im| (low-precision MFMA scaling)
    GroupState* d_state = nullptr;     // graph replays: current launch group
    hipStream_t cap_stream = nullptr;  // private stream for graph capture
    // captured graphs: gexec[0] runs one launch group, gexec[1] g_many
    // consecutive groups (the group index advances on the device)
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int g_many = 0;
    hipEvent_t g_done = nullptr;       // recorded after the last replays
    void* g_ws[2] = {nullptr, nullptr};    // buffers each graph was captured with
    double* g_acc[2] = {nullptr, nullptr};
    uint64_t graph_replays = 0;        // statistics: launch groups replayed from graphs
    uint64_t graph_launches = 0;       // and graph launches
    Profiler prof;
    // concurrent lanes of launch groups (set_lanes): lane 0 is this state on
    // the caller's stream, lanes 1 .. n_lanes - 1 are made on first use
    int n_lanes = 1;
    hipEvent_t fork = nullptr;
    std::vector<std::unique_ptr<Lane>> lanes;
};

// An extra lane: its own stream, workspace slice, max slots, group state,
// graphs and float64 accumulator; the plan memory (leaves and slice-invariant
// tensors) is the plan's, read only.
struct Lane {
    DeviceState d;
    hipStream_t stream = nullptr;
    hipEvent_t join = nullptr;
    double* acc = nullptr;
    uint64_t acc_n = 0;   // complex128 entries
};

struct Group {
    uint64_t slice_base;          // slice id with the batch bits zero
    uint64_t beta0, beta1;        // batch slots [beta0, beta1) when mask is empty
    std::vector<uint32_t> mask;   // explicit batch slots (slice lists)
};

std::string prepare(Plan& p, DeviceState& d, hipStream_t s);
// Kernel configurations (kernel, tile) that can run step `step` (index into
// p.steps), and forcing one of them (drops a captured graph).
std::vector<std::pair<int, int>> step_candidates(const Plan& p, int step);
std::string set_step_kernel(Plan& p, DeviceState& d, int step, int kernel, int tile);
// Replace the data of a leaf (natural order of its legs) in prepared plan memory.
std::string upload_leaf(Plan& p, DeviceState& d, int leaf, std::vector<cd> data, hipStream_t s);
std::string run_groups(Plan& p, DeviceState& d, void* ws, double* acc, const std::vector<Group>& groups,
                       hipStream_t s);
// Workspace bytes between lanes (stats.workspace_bytes rounded up to 256) and
// the bytes n lanes need.
uint64_t lane_stride(const Plan& p);
uint64_t lanes_workspace_bytes(const Plan& p, int n);
// Number of lanes of later calls (1 .. kMaxLanes); fewer releases the extra
// lanes (after their work has finished).
constexpr int kMaxLanes = 8;
std::string set_lanes(DeviceState& d, int n);
// run_groups over as many lanes as are set and fit in ws_bytes: the groups
// are split into contiguous runs, one per lane, run concurrently; the
// caller's stream waits for every lane and adds the lanes' sums to acc in
// lane order.  One lane (run_groups itself) while step timing is on, for
// slice lists, or with fewer than two groups per lane.
std::string run_lanes(Plan& p, DeviceState& d, void* ws, size_t ws_bytes, double* acc,
                      const std::vector<Group>& groups, hipStream_t s);
void release(DeviceState& d);
std::string profile_enable(Plan& p, DeviceState& d, bool on);
std::string profile_harvest(DeviceState& d);
std::string autotune(Plan& p, DeviceState& d, void* ws, double* acc, const char* cache_path, int reps, int& n_tuned,
                     hipStream_t s);

int storage_of(tn_precision p);

}  // namespace tn
