// Profile records (counter-based and context-based, paper Sec. III-C).
#pragma once
#include <vector>

#include "../../include/qops.h"

struct qops_profile {
    int n = 0;
    int prec = 0;
    double total = 0;                       // sum of pass times (s)
    std::vector<qops_pass_record> recs;     // one per pass, in execution order
    std::vector<float> feats;               // cost-model features, 64 per pass
    std::vector<int32_t> lcount, pcount;    // [kind][qubit] gate counters
};
