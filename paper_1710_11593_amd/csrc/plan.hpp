// Plan selection (plan.hip): leaf size and dense/FFT crossover of a handle.
#pragma once

#include <stdint.h>

#include <string>

namespace fs {

struct PlanEntry {
    int precision, equation, m_max, leaf, crossover;
};

struct Plan {
    int leaf;       // leaf size L
    int crossover;  // largest dense half-size s*; < 0: FFT at every level
    int source;     // FRACSOLVE_PLAN_OPTIONS / _CACHE / _BUILTIN
};

// Path of the plan cache file ("" if none can be formed).
std::string plan_cache_path();

// The plan for a handle of this precision and equation whose widest instance
// has mmax points; leaf_opt / crossover_opt are the options (0 = choose).
Plan resolve_plan(int precision, int equation, int64_t mmax, int leaf_opt, int crossover_opt);

}  // namespace fs
