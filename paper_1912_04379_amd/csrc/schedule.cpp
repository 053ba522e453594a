// schedule.cpp -- the list schedule of grouped plans.  Host code only, free
// of HIP (rules.hpp).
#include <functional>
#include <queue>
#include <utility>
#include <vector>

#include "rules.hpp"

namespace mgemm {

std::vector<uint32_t> lpt_schedule(const std::vector<double>& cost_in_order, uint32_t G) {
    std::vector<uint32_t> owner(cost_in_order.size());
    if (G == 0) G = 1;
    // (assigned cost, work-group): the least-loaded on top, ties to the
    // lowest number.
    using Load = std::pair<double, uint32_t>;
    std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
    for (uint32_t w = 0; w < G; ++w) heap.push(Load{0.0, w});
    for (size_t i = 0; i < cost_in_order.size(); ++i) {
        Load l = heap.top();
        heap.pop();
        owner[i] = l.second;
        l.first += cost_in_order[i];
        heap.push(l);
    }
    return owner;
}

}  // namespace mgemm
