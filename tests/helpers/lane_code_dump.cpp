// Prints the matrix and the check order compiled into the one-lane layered
// kernel (lane_code.h): a line "rows" then one line per check with its
// variables, then a line "order" with the checks in the order the kernel
// updates them and the number of layers.
#include <cstdio>

#include "lane_code.h"

int main() {
    using namespace sagms::lane;
    std::printf("rows %d %d %d\n", kL, kN, kDC);
    for (int c = 0; c < kL; ++c) {
        for (int k = 0; k < kDC; ++k) std::printf(k ? " %d" : "%d", kRows.var[c][k]);
        std::printf("\n");
    }
    std::printf("order %d", kOrder.layers);
    for (int i = 0; i < kL; ++i) std::printf(" %d", kOrder.check[i]);
    std::printf("\n");
    return 0;
}
