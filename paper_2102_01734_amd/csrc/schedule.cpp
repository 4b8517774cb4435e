// schedule.cpp -- static distribution of formal-solution work over the
// persistent workgroups of one launch.
//
// A work item is (wavelength, direction): all characteristics of that
// direction for that wavelength, swept through the grid by one workgroup.
// Its cost is the template length M_d (visits per characteristic), which
// varies by ~10x between steep and shallow directions (the load imbalance the
// paper reports for the periodic box, Sec. 4.1).  Each workgroup writes its
// J / Lambda* contributions into partial-sum slots that only it owns; the
// reduction adds the slots of a wavelength in a fixed order, so results do
// not depend on timing.
//
// * ray bundles: when a direction's rays are split into n_bundles bundles,
//   workgroup w sweeps bundle w mod n_bundles, and each class of workgroups
//   receives every item, distributed as below.
// * one wavelength, class size a multiple of 4 (the dispatcher places
//   workgroup i on XCD i mod 8): directions
//   that sweep downwards go to the workgroups of XCDs 0-3, upward ones to
//   XCDs 4-7, and each sign's directions are dealt in rounds of equal cost
//   (sorted by cost, one item per workgroup per round, heaviest item to the
//   least loaded workgroup).  The 32 CUs of an XCD then sweep directions of
//   similar length through similar layers at the same time and share the
//   opacity/source data in their L2.
// * batch <= workgroups: every wavelength gets its own group of workgroups
//   (sizes differ by at most one) and its directions are spread over them by
//   longest-processing-time-first; one slot per workgroup.
// * batch >  workgroups: items are laid out wavelength-major and cut into
//   n_wg contiguous runs of equal cost; a workgroup opens a new slot whenever
//   its run enters a new wavelength.
#include <algorithm>
#include <numeric>
#include <queue>
#include <vector>

#include "rt_internal.hpp"

namespace rt3d {

// One class of workgroups (those sweeping the same ray bundle) gets every
// (wavelength, direction) item; `wgs` are the class's workgroup ids.
static void schedule_class(const BoxGeometry &g, const std::vector<int32_t> &lambdas, const std::vector<int> &order,
                           const std::vector<int> &wgs, std::vector<std::vector<WorkItem>> &per_wg,
                           std::vector<std::vector<int32_t>> &slots_of_lambda, int &slot)
{
    const int nl = (int)lambdas.size();
    const int nd = (int)order.size();
    const int n_wg = (int)wgs.size();
    const bool xcd_rounds = nl == 1 && n_wg % 4 == 0 && nd >= n_wg;
    if (xcd_rounds) {
        std::vector<int64_t> load(per_wg.size(), 0);
        std::vector<int> used;
        for (int sign = 0; sign < 2; ++sign) {
            std::vector<int> dirs;
            for (int di : order)  // already sorted by decreasing cost
                if ((g.dirs[di].mu < 0.0) == (sign == 0)) dirs.push_back(di);
            std::vector<int> half;  // XCDs 0-3 for downward sweeps, 4-7 for upward
            for (int w : wgs)
                if (((w % 8) < 4) == (sign == 0)) half.push_back(w);
            if (half.empty()) half = wgs;
            const int k = (int)half.size();
            for (size_t r0 = 0; r0 < dirs.size(); r0 += k) {
                const size_t r1 = std::min(dirs.size(), r0 + (size_t)k);
                std::vector<int> by_load(half);
                std::stable_sort(by_load.begin(), by_load.end(), [&](int a, int b) { return load[a] < load[b]; });
                for (size_t t = r0; t < r1; ++t) {
                    const int w = by_load[t - r0];
                    per_wg[w].push_back({lambdas[0], dirs[t], w, per_wg[w].empty() ? 1 : 0});
                    load[w] += g.dirs[dirs[t]].M;
                }
            }
        }
        for (int w : wgs)
            if (!per_wg[w].empty()) slots_of_lambda[0].push_back(w);
        slot = std::max(slot, (int)per_wg.size());
    } else if (nl <= n_wg) {
        // workgroups per wavelength: as even as possible, but never more than directions
        std::vector<int> cnt(nl, n_wg / nl);
        for (int i = 0; i < n_wg % nl; ++i) cnt[i]++;
        for (int i = 0; i < nl; ++i) cnt[i] = std::max(1, std::min(cnt[i], nd));
        int next = 0;  // next workgroup of the class
        for (int li = 0; li < nl; ++li) {
            const int k = cnt[li];
            // LPT: longest direction to the least loaded workgroup of this wavelength
            using P = std::pair<int64_t, int>;  // (load, local wg), min-heap
            std::priority_queue<P, std::vector<P>, std::greater<P>> heap;
            std::vector<std::vector<WorkItem>> local(k);
            for (int w = 0; w < k; ++w) heap.push({0, w});
            for (int di : order) {
                P top = heap.top();
                heap.pop();
                local[top.second].push_back({lambdas[li], di, 0, 0});
                heap.push({top.first + g.dirs[di].M, top.second});
            }
            for (int w = 0; w < k; ++w) {
                if (local[w].empty()) continue;
                const int wg = wgs[(next++) % n_wg];
                for (auto &it : local[w]) it.slot = slot;
                local[w][0].first = 1;
                slots_of_lambda[li].push_back(slot);
                ++slot;
                for (auto &it : local[w]) per_wg[wg].push_back(it);
            }
        }
    } else {
        // contiguous equal-cost runs over the wavelength-major item list
        int64_t per_lambda = 0;
        for (int di : order) per_lambda += g.dirs[di].M;
        const int64_t total = per_lambda * nl;
        int64_t acc = 0;
        int v = 0;  // class-local workgroup
        int cur_lambda = -1;
        for (int li = 0; li < nl; ++li) {
            for (int di : order) {
                // move to the next workgroup once this one has its share
                const int64_t target = (total * (v + 1)) / n_wg;
                if (acc >= target && v + 1 < n_wg && !per_wg[wgs[v]].empty()) {
                    ++v;
                    cur_lambda = -1;
                }
                auto &list = per_wg[wgs[v]];
                if (cur_lambda != li) {
                    slots_of_lambda[li].push_back(slot);
                    list.push_back({lambdas[li], di, slot, 1});
                    ++slot;
                    cur_lambda = li;
                } else {
                    list.push_back({lambdas[li], di, slot - 1, 0});
                }
                acc += g.dirs[di].M;
            }
        }
    }
}

void build_schedule(const BoxGeometry &g, const std::vector<int32_t> &lambdas, int n_wg, Schedule &out,
                    const std::vector<int32_t> *subset, int n_bundles)
{
    out = Schedule();
    const int nl = (int)lambdas.size();
    std::vector<int> order;
    if (subset) {
        order.assign(subset->begin(), subset->end());
    } else {
        order.resize(g.dirs.size());
        std::iota(order.begin(), order.end(), 0);
    }
    const int nd = (int)order.size();
    out.slot_begin.assign(nl + 1, 0);
    if (nl == 0 || nd == 0 || n_wg <= 0 || n_bundles < 1 || n_wg < n_bundles) {
        out.n_wg = 0;
        out.wg_begin.assign(1, 0);
        return;
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return g.dirs[a].M > g.dirs[b].M; });

    std::vector<std::vector<WorkItem>> per_wg(n_wg);
    std::vector<std::vector<int32_t>> slots_of_lambda(nl);
    int slot = 0;
    for (int b = 0; b < n_bundles; ++b) {
        std::vector<int> wgs;
        for (int w = b; w < n_wg; w += n_bundles) wgs.push_back(w);
        schedule_class(g, lambdas, order, wgs, per_wg, slots_of_lambda, slot);
    }
    // slots are numbered by workgroup id in the XCD-rounds case and densely otherwise
    int n_slots = 0;
    for (int li = 0; li < nl; ++li)
        for (int s : slots_of_lambda[li]) n_slots = std::max(n_slots, s + 1);
    out.n_slots = n_slots;
    out.n_wg = n_wg;
    out.wg_begin.assign(out.n_wg + 1, 0);
    for (int w = 0; w < out.n_wg; ++w) {
        out.wg_begin[w + 1] = out.wg_begin[w] + (int32_t)per_wg[w].size();
        out.items.insert(out.items.end(), per_wg[w].begin(), per_wg[w].end());
    }
    for (int li = 0; li < nl; ++li) {
        out.slot_begin[li + 1] = out.slot_begin[li] + (int32_t)slots_of_lambda[li].size();
        out.slot_ids.insert(out.slot_ids.end(), slots_of_lambda[li].begin(), slots_of_lambda[li].end());
    }
}

std::vector<int32_t> shard_directions(const BoxGeometry &g, int n_shards, int shard)
{
    const int nd = (int)g.dirs.size();
    std::vector<int> order(nd);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return g.dirs[a].M > g.dirs[b].M; });
    using P = std::pair<int64_t, int>;  // (visits, shard), min-heap
    std::priority_queue<P, std::vector<P>, std::greater<P>> heap;
    for (int s = 0; s < n_shards; ++s) heap.push({0, s});
    std::vector<int32_t> out;
    for (int di : order) {
        P top = heap.top();
        heap.pop();
        if (top.second == shard) out.push_back(di);
        heap.push({top.first + g.dirs[di].M, top.second});
    }
    std::sort(out.begin(), out.end());
    return out;
}

}  // namespace rt3d
