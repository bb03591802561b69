// symitems.hpp -- the work item of the symmetric all-pairs sum, shared by the
// kernels (pairsym.hpp) and the host code that builds the item lists
// (worksplit.hpp).  Plain C++: no device code.
#pragma once

namespace odk {

// Target tile rows that share one pass over the sources (sym_rows).
constexpr int kSymRows = 3;

// rows == 1: target tile row I against source tiles [J0, J1) (sym_item), of
// each source tile only the 64-ion sub-tiles [st0, st1) (0..4: the whole
// tile); rows == kSymRows: target tile rows I .. I + kSymRows - 1 together
// (sym_rows), whole tiles.
struct SymItem {
    int I, J0, J1, rows, st0, st1;
};

}  // namespace odk
