// Learned cost model internals shared with the plan pricer.
#pragma once
#include "../../include/qops.h"

namespace qops {
// Evaluates the trained network on the host (FP32) for plan pricing.
void mlp_predict_host(const qops_model* m, const float* features, int rows, float* out);
}  // namespace qops
