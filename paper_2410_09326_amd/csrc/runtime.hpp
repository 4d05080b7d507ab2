// Internal runtime structures shared by the ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/qops.h"
#include "planner.hpp"

struct qops_sim {
    int n = 0;
    int prec = 0;
    void* state = nullptr;
    bool owned = false;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    int device = 0;                   // HIP device current at creation (owner of the state)
    std::vector<int> l2p;             // logical qubit -> physical bit
    double* scratch = nullptr;        // reductions / readout staging
    size_t scratch_doubles = 0;
    qops::Plan* last_plan = nullptr;  // kept alive until the next apply / destroy
    int grid_cap = 0;                 // work-group limit of state passes (0 = the kernels' own)
    std::vector<hipEvent_t> events;   // per-pass timing events of profiled runs (reused)
};

struct qops_plan {
    qops::Plan p;
};

namespace qops {

int32_t set_error(int32_t code, const std::string& msg);
int32_t hip_fail(hipError_t e, const char* what);
size_t amp_size(int prec);
int32_t upload_plan(Plan& p);
void free_plan_device(Plan& p);
int32_t launch_pass(qops_sim* h, const Plan& p, const PassPlan& pp);
int32_t check_plan_matches(qops_sim* h, const Plan& p);
int32_t run_plan(qops_sim* h, Plan& p);
int32_t ensure_scratch(qops_sim* h, size_t doubles);
PlanParams params_from(const qops_plan_opts* o, int n, int prec);

// Plans a gate list; PROFILED / LEARNED modes price candidate plans with the
// profile's cost table or the trained model and keep the cheapest.
int32_t build_priced_plan(int n, int prec, const int32_t* l2p, const qops_gate* g, size_t ng,
                          const qops_plan_opts* opts, Plan& out);

}  // namespace qops
