// Host check of the symmetric sum's work split (csrc/worksplit.hpp): for
// every tile count T tried, the items built by sym_items_of must take every
// unordered pair of tiles (a <= b), and each of its four 64-ion source
// sub-tiles, exactly once, under the loops the kernels run for an item:
//   rows == 1:  target row I against sub-tiles [st0, st1) of the source tiles J in [J0, J1);
//   rows == R:  when J0 == I, each row I + r first against tiles I + r .. I + R - 1,
//               then every row I .. I + R - 1 against tiles [max(J0, I + R), J1).
// Also checks that every item is well formed, that a grouped item starting at
// its own rows reaches past them, that sym_items orders the same items
// longest first, and the same coverage for the one-row split (every item one
// target row) and for a smaller items target.  Exit status 0 when all hold.
#include <cstdio>
#include <vector>

#include "worksplit.hpp"

static int check(int T, bool one_row, double target = kSymItemsTarget)
{
    const std::vector<odk::SymItem> items = sym_items_of(T, one_row, target);
    std::vector<unsigned char> seen((size_t)T * T, 0);     // bit st: sub-tile st taken
    auto take = [&](int a, int b, int st0 = 0, int st1 = 4) {
        if (a < 0 || b < a || b >= T) return false;
        const unsigned char m = (unsigned char)(((1u << st1) - 1u) & ~((1u << st0) - 1u));
        unsigned char& s = seen[(size_t)a * T + b];
        if (s & m) return false;
        s |= m;
        return true;
    };
    for (const odk::SymItem& it : items) {
        const int R = it.rows;
        if (!(R == 1 || R == odk::kSymRows) || it.I < 0 || it.I + R > T || it.J0 < it.I || it.J1 <= it.J0 ||
            it.J1 > T || it.st0 < 0 || it.st1 > 4 || it.st0 >= it.st1 || (R != 1 && (it.st0 || it.st1 != 4))) {
            std::printf("T=%d: malformed item (%d, %d, %d, %d, %d, %d)\n", T, it.I, it.J0, it.J1, R, it.st0,
                        it.st1);
            return 1;
        }
        if (one_row && R != 1) return std::printf("T=%d: a grouped item in the one-row split\n", T), 1;
        if (R == 1) {
            for (int J = it.J0; J < it.J1; ++J)
                if (!take(it.I, J, it.st0, it.st1)) return std::printf("T=%d: pair (%d, %d) twice\n", T, it.I, J), 1;
            continue;
        }
        int J0 = it.J0;
        if (J0 == it.I) {
            if (it.J1 < it.I + R) return std::printf("T=%d: grouped item ends inside its rows\n", T), 1;
            for (int r = 0; r < R; ++r)
                for (int J = it.I + r; J < it.I + R; ++J)
                    if (!take(it.I + r, J)) return std::printf("T=%d: pair (%d, %d) twice\n", T, it.I + r, J), 1;
            J0 = it.I + R;
        }
        for (int r = 0; r < R; ++r)
            for (int J = J0; J < it.J1; ++J)
                if (!take(it.I + r, J)) return std::printf("T=%d: pair (%d, %d) twice\n", T, it.I + r, J), 1;
    }
    for (int a = 0; a < T; ++a)
        for (int b = a; b < T; ++b)
            if (seen[(size_t)a * T + b] != 0xF) return std::printf("T=%d: pair (%d, %d) missing\n", T, a, b), 1;
    if (one_row || target != kSymItemsTarget) return 0;   // the launch order is checked for the default split
    // the launch order: the same items, most work first
    const std::vector<odk::SymItem> sorted = sym_items(T);
    if (sorted.size() != items.size()) return std::printf("T=%d: sorted list differs in size\n", T), 1;
    for (size_t k = 1; k < sorted.size(); ++k)
        if (sym_item_cost(sorted[k]) > sym_item_cost(sorted[k - 1]))
            return std::printf("T=%d: items not longest first\n", T), 1;
    return 0;
}

int main()
{
    int fails = 0, grouped = 0, single = 0, subtiles = 0;
    std::vector<int> Ts;
    for (int T = 1; T <= 700; ++T) Ts.push_back(T);
    for (int T : {1021, 1024, 1025, 2048, 4095, 4096, 4097}) Ts.push_back(T);
    for (int T : Ts) {
        fails += check(T, false) + check(T, true) + check(T, false, 4096.0) + check(T, true, 4096.0);
        const std::vector<odk::SymItem> v = sym_items_of(T);
        (v.size() && v[0].rows == odk::kSymRows) ? ++grouped : ++single;
        subtiles += v.size() && v[0].st1 - v[0].st0 == 1;
    }
    std::printf("%zu tile counts checked (%d split into grouped rows, %d into single rows, %d of them into "
                "sub-tiles), %d failures\n", Ts.size(), grouped, single, subtiles, fails);
    return fails ? 1 : 0;
}
