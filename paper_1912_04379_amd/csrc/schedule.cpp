// schedule.cpp -- the list schedule of grouped plans.  Host code only, free
// of HIP (rules.hpp).
#include <algorithm>
#include <cmath>
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

std::vector<std::vector<std::pair<uint32_t, uint32_t>>> queue_partition(
    const std::vector<uint32_t>& ntiles, const std::vector<double>& tile_cost, uint32_t nq) {
    if (nq == 0) nq = 1;
    double total = 0.0;
    for (size_t i = 0; i < ntiles.size(); ++i) total += ntiles[i] * tile_cost[i];
    const double target = total / nq;
    // Problems costing more than one queue's share are cut into contiguous
    // runs of tiles, so that one large problem still spreads over queues.
    struct Chunk {
        uint32_t problem, first, count;
        double cost;
    };
    std::vector<Chunk> chunks;
    for (size_t i = 0; i < ntiles.size(); ++i) {
        const uint32_t n = ntiles[i];
        if (n == 0) continue;
        const double c = n * tile_cost[i];
        uint32_t k = target > 0.0 && c > target ? (uint32_t)std::ceil(c / target) : 1u;
        if (k > n) k = n;
        const uint32_t per = (n + k - 1) / k;
        for (uint32_t f = 0; f < n; f += per) {
            const uint32_t cnt = std::min(per, n - f);
            chunks.push_back(Chunk{(uint32_t)i, f, cnt, cnt * tile_cost[i]});
        }
    }
    std::stable_sort(chunks.begin(), chunks.end(),
                     [](const Chunk& a, const Chunk& b) { return a.cost > b.cost; });
    std::vector<double> costs(chunks.size());
    for (size_t c = 0; c < chunks.size(); ++c) costs[c] = chunks[c].cost;
    const std::vector<uint32_t> owner = lpt_schedule(costs, nq);
    // Each queue: its tiles, costliest first (ties keep chunk, then tile order).
    std::vector<std::vector<std::pair<double, std::pair<uint32_t, uint32_t>>>> q(nq);
    for (size_t c = 0; c < chunks.size(); ++c)
        for (uint32_t t = 0; t < chunks[c].count; ++t)
            q[owner[c]].push_back({tile_cost[chunks[c].problem],
                                   {chunks[c].problem, chunks[c].first + t}});
    std::vector<std::vector<std::pair<uint32_t, uint32_t>>> out(nq);
    for (uint32_t i = 0; i < nq; ++i) {
        std::stable_sort(q[i].begin(), q[i].end(),
                         [](const auto& a, const auto& b) { return a.first > b.first; });
        out[i].reserve(q[i].size());
        for (const auto& e : q[i]) out[i].push_back(e.second);
    }
    return out;
}

}  // namespace mgemm
