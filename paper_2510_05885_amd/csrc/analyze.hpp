// analyze.hpp — host symbolic analysis entry point.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "plan.hpp"

namespace ncl {

struct SysInput {
    int n = 0, m = 0;
    const int32_t *Wp = nullptr, *Wi = nullptr, *Jp = nullptr, *Jj = nullptr;
};

// Builds the plan of `sys` (one system, or several independent ones forming a
// block-diagonal matrix) for form 0 (condensed) or 1 (stabilized).
// ordering: 0 nested dissection, 1 natural, 2 user (user_perm).
// Returns 0 or a negative NCL error code with a message in err.
int build_plan(Plan& P, int form, const std::vector<SysInput>& sys, int ordering, const int32_t* user_perm,
               const PlanConfig& cfg, std::string& err);

}  // namespace ncl
