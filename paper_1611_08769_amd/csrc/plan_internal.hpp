// A compiled encrypted-FFT plan as shared by the plan ABI and the server.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/sfft.h"
#include "device.hpp"
#include "schedule.hpp"

namespace sfft {

struct PlanCore {
    sfft_shape shape{};
    sfft_params params{};
    Geo geo{};
    ProdCfg cfg{};
    Schedule sched;
    sfft_plan_info info{};
    int64_t points = 0;  // FFT points (len or len^2)
    ProdItem* d_prods = nullptr;
    LinItem* d_lins = nullptr;
    LinItem* d_final = nullptr;
    // per step s (levels, then the output pass): the step's workgroups and the
    // bit-MACs (products x Nct^3) of steps s.. to the end
    std::vector<int64_t> step_blocks;
    std::vector<double> work_from;
    // the plan's launch sequence captured for one set of buffers (sfft_execute_graph)
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    const void* graph_in = nullptr;
    const void* graph_out = nullptr;
    const void* graph_ws = nullptr;
    // whole-plan persistent execution (sfft_execute_persistent): the level
    // and pass tables on the device, the barrier words, built on first use
    int64_t* d_persist = nullptr;
    uint32_t* d_bar = nullptr;
    // product-kernel timing (sfft_plan_time_products): event pairs recorded
    // around each level's product kernel by sfft_execute_steps while on
    mutable bool time_products = false;
    mutable std::vector<std::pair<hipEvent_t, hipEvent_t>> prod_events;

    int64_t ct_words() const { return (int64_t)geo.nct * geo.W; }
    // workspace: the slots, then (where a matrix-core tiling serves the
    // geometry) the chunk-layout copies of one level's right operands
    int64_t slot_bytes() const { return sched.n_slots * ct_words() * 4; }
    int64_t rt_bytes() const { return sched.max_level_products * rt_item_bytes(geo); }
    int64_t ws_bytes() const { return slot_bytes() + rt_bytes(); }
    PlanCore() = default;
    PlanCore(const PlanCore&) = delete;
    PlanCore& operator=(const PlanCore&) = delete;
    ~PlanCore();
};

// Compile (and, with upload, copy the work tables to the device).
// ws_limit > 0 bounds the workspace (levels by list scheduling within it).
int plan_core_build(const sfft_shape* shape, const sfft_params* params, bool upload, PlanCore* out,
                    int64_t ws_limit = 0);

}  // namespace sfft

// The compiled core of a public plan handle (defined with the ABI).
const sfft::PlanCore* plan_core_of(const struct sfft_plan* plan);

// status helpers shared by the ABI translation units (set sfft_last_error)
int sfft_fail(int code, const std::string& msg);
int sfft_hip_fail(hipError_t e, const char* where);
