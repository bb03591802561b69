// worksplit.hpp -- host side: how the symmetric all-pairs sum of one system
// is cut into work items (pair_sym_kernel, pair_sym_batch_kernel).  Kept
// apart from the rest of the host code because, with the kernels, it fixes
// what the pair phase reads and writes.
#pragma once

#include <algorithm>
#include <cmath>
#include <vector>

#include "symitems.hpp"

namespace {

constexpr double kSymItemsTarget = 65536.0;    // work items of the symmetric sum
constexpr double kSymMinGroupedItems = 2048.0; // fewer grouped items: one target row per item
constexpr double kSymMinItems = 512.0;         // fewer one-tile items: one item per 64-ion sub-tile

// Work items of the symmetric sum of one system of T tiles: groups of
// kSymRows target tile rows, each group with runs of at most C source tiles
// from its first row on (rows left over at the end alone), C chosen for about
// kSymItemsTarget items.  Where grouping leaves fewer than kSymMinGroupedItems
// items (small systems, too few to fill the chip), one target row per item
// instead; where even one tile pair per item leaves fewer than kSymMinItems
// (a few thousand ions), each tile pair is cut into its four 64-ion source
// sub-tiles, so that a step's pair sum is not one long chain per block.  The
// split depends on T only, so a system's sums are grouped the same way alone
// and in a batch.  one_row: one target row per item at every size; target:
// the number of items aimed at (batch options; both change the FP32 partial
// sums that each item flushes).
std::vector<odk::SymItem> sym_items_of(int T, bool one_row = false, double target = kSymItemsTarget)
{
    constexpr int R = odk::kSymRows;
    const double pairs = 0.5 * (double)T * (T + 1);
    std::vector<odk::SymItem> v;
    const int C = (int)std::max((double)R, std::ceil(pairs / (R * target)));
    int I = 0;
    for (; I + R <= T; I += R)
        for (int J0 = I; J0 < T; J0 += C) v.push_back({I, J0, std::min(J0 + C, T), R, 0, 4});
    for (; I < T; ++I) v.push_back({I, I, T, 1, 0, 4});
    if ((double)v.size() >= kSymMinGroupedItems && !one_row) return v;
    v.clear();
    const int C1 = (int)std::max(1.0, std::ceil(pairs / target));
    const bool sub = C1 == 1 && pairs < kSymMinItems;
    for (I = 0; I < T; ++I)
        for (int J0 = I; J0 < T; J0 += C1) {
            if (!sub) {
                v.push_back({I, J0, std::min(J0 + C1, T), 1, 0, 4});
                continue;
            }
            for (int st = 0; st < 4; ++st) v.push_back({I, J0, J0 + 1, 1, st, st + 1});
        }
    return v;
}

// Work of an item: target rows times 64-ion source sub-tiles.
inline long long sym_item_cost(int rows, int J0, int J1, int st0, int st1)
{
    return (long long)rows * (J1 - J0) * (st1 - st0);
}
inline long long sym_item_cost(const odk::SymItem& a) { return sym_item_cost(a.rows, a.J0, a.J1, a.st0, a.st1); }

// Longest items first, so that the short ones fill the tail.
std::vector<odk::SymItem> sym_items(int T)
{
    std::vector<odk::SymItem> v = sym_items_of(T);
    std::stable_sort(v.begin(), v.end(), [](const odk::SymItem& a, const odk::SymItem& b) {
        return sym_item_cost(a) > sym_item_cost(b);
    });
    return v;
}

}  // namespace
