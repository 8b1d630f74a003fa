// The code compiled into the one-lane-per-frame layered decoder
// (layered_lane.hip): the generalized-bicycle code of Section V with
// circulant size l = 63, a(x) = 1 + x + x^14 + x^16 + x^22 and
// b(x) = 1 + x^3 + x^13 + x^20 + x^42 (the [[126, 28]] code of the paper's
// l = 63 experiments), decoded with H_Z = [B^T | A^T] as sagms_build_gb
// builds it: row c has ones at (c - b_t) mod l and l + (c - a_t) mod l.
//
// Its rows and its layered check order are constant expressions, so the
// kernel addresses every posterior and check output by a register name.
// The host compares a graph's rows with these before it selects the kernel
// (layers.cpp), so the kernel only ever runs the matrix it was compiled for.
#pragma once

#include <cstdint>

namespace sagms {
namespace lane {

constexpr int kL = 63;       // checks (rows of H_Z)
constexpr int kN = 2 * kL;   // variables
constexpr int kDC = 10;      // check degree
constexpr int kTerms = 5;    // terms of a(x) and of b(x)
constexpr int kA[kTerms] = {0, 1, 14, 16, 22};
constexpr int kB[kTerms] = {0, 3, 13, 20, 42};

struct Rows {
    int var[kL][kDC];  // variables of check c; edge order is free (the check update is symmetric)
};

constexpr Rows make_rows() {
    Rows r{};
    for (int c = 0; c < kL; ++c)
        for (int t = 0; t < kTerms; ++t) {
            r.var[c][t] = ((c - kB[t]) % kL + kL) % kL;
            r.var[c][kTerms + t] = kL + ((c - kA[t]) % kL + kL) % kL;
        }
    return r;
}

// Checks in (layer, index) order for the first-fit layers in ascending check
// index (check c joins the first layer none of whose checks shares a
// variable with it).  Updating the checks one after another in this order
// gives every variable its checks in layer order, so the results equal those
// of the layer-by-layer schedule.
struct Order {
    int check[kL];
    int layers;
};

constexpr Order make_order(const Rows& r) {
    Order o{};
    uint64_t used[kL][2] = {};
    int layer_of[kL] = {};
    int nl = 0;
    for (int c = 0; c < kL; ++c) {
        uint64_t mine[2] = {0, 0};
        for (int k = 0; k < kDC; ++k) mine[r.var[c][k] >> 6] |= 1ull << (r.var[c][k] & 63);
        int l = 0;
        while (l < nl && ((used[l][0] & mine[0]) | (used[l][1] & mine[1])) != 0) ++l;
        if (l == nl) ++nl;
        used[l][0] |= mine[0];
        used[l][1] |= mine[1];
        layer_of[c] = l;
    }
    int k = 0;
    for (int l = 0; l < nl; ++l)
        for (int c = 0; c < kL; ++c)
            if (layer_of[c] == l) o.check[k++] = c;
    o.layers = nl;
    return o;
}

constexpr Rows kRows = make_rows();
constexpr Order kOrder = make_order(kRows);

}  // namespace lane
}  // namespace sagms
