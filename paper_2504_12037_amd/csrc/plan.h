// Width-set planner (Sec. 2, finding the width set): a greedy min-fill
// elimination order pi of the whole interaction graph, dynamic slicing of
// the index shared by the most widest intermediates until the width of pi
// restricted to R is within the bound, then indices put back from W in key
// order wherever the bound still holds.  Host only.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tnvan.h"

namespace tnvan {

struct PlanResult {
  std::vector<int32_t> W;       // ascending id
  std::vector<int32_t> order;   // the order of R
  std::vector<int32_t> pi;      // greedy order of all vertices
  int32_t width = 0;            // width of `order`
};

constexpr int32_t kPlanMaxSpins = 16384;

// key: a permutation of 0..n-1 (ties and the re-adding order), or empty for
// the identity.  Returns TNVAN_E_INVALID with a message on bad input.
tnvan_status plan_width_set(int32_t n, const std::vector<int32_t> &ei,
                            const std::vector<int32_t> &ej, int32_t w_u,
                            const std::vector<int32_t> &key, bool regreedy,
                            PlanResult &out, std::string &msg);

}  // namespace tnvan
