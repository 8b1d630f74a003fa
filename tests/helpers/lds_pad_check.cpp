// Checks the placement of the decoder's padding lanes (lds_pad.h) on the
// host: every padding lane ends on a word of its pool, all padding lanes of
// one half-wavefront share one word, and that word's bank is one the half's
// real lanes leave free, so padding adds no bank-conflict cycle under the
// LDS model of two halves of 32 lanes on 32 banks.  Cases: the l = 63 GB
// code's check-side gathers (a rotation of 63 posteriors plus one padding
// lane), its variable-side tail (two padding lanes), an all-padding row, and
// random rows.  Prints "ok <cases>" or the first failing case.
#include <cstdio>
#include <map>
#include <random>
#include <set>
#include <vector>

#include "lds_pad.h"

using namespace sagms;

// extra cycles of one half: the largest number of distinct words in one bank, minus 1
static int half_extra(const std::vector<uint32_t>& row, int h) {
    std::map<int, std::set<uint32_t>> per;
    for (int l = 32 * h; l < 32 * h + 32; ++l) per[row[l] % kLdsBanks].insert(row[l]);
    size_t d = 0;
    for (auto& kv : per) d = kv.second.size() > d ? kv.second.size() : d;
    return (int)d - 1;
}

// real-lane-only extra cycles of one half (padding lanes ignored)
static int half_extra_real(const std::vector<uint32_t>& row, int h) {
    std::map<int, std::set<uint32_t>> per;
    for (int l = 32 * h; l < 32 * h + 32; ++l)
        if (row[l] != kPadLane) per[row[l] % kLdsBanks].insert(row[l]);
    size_t d = 1;
    for (auto& kv : per) d = kv.second.size() > d ? kv.second.size() : d;
    return (int)d - 1;
}

static bool check_row(const std::vector<uint32_t>& before, uint32_t pool) {
    std::vector<uint32_t> after = before;
    place_padding(after, pool);
    for (int h = 0; h < 2; ++h) {
        uint32_t word = kPadLane;
        int real = 0;
        for (int l = 32 * h; l < 32 * h + 32; ++l) {
            if (before[l] != kPadLane) {
                ++real;
                if (after[l] != before[l]) return false;  // real lanes untouched
                continue;
            }
            if (after[l] < pool || after[l] >= pool + 64) return false;
            if (word != kPadLane && after[l] != word) return false;
            word = after[l];
        }
        if (word == kPadLane) continue;
        // with at most 31 real lanes a free bank exists: no added cycle
        if (real < 32 && half_extra(after, h) != half_extra_real(before, h)) return false;
        for (int l = 32 * h; l < 32 * h + 32; ++l)
            if (before[l] != kPadLane && before[l] % kLdsBanks == word % kLdsBanks) return false;
    }
    return true;
}

int main() {
    int cases = 0;
    const uint32_t post0 = 704, pool_inf = 832, pool_zero = 640;
    // check-side gathers of the l = 63 code: lane c < 63 reads the posterior
    // of variable (c - b) mod 63 of one block, lane 63 pads
    for (int block = 0; block < 2; ++block)
        for (int b = 0; b < 63; ++b) {
            std::vector<uint32_t> row(64, kPadLane);
            for (int c = 0; c < 63; ++c) row[c] = post0 + 63 * block + (uint32_t)((c - b + 63) % 63);
            if (!check_row(row, pool_inf)) { printf("fail cn block %d b %d\n", block, b); return 1; }
            ++cases;
        }
    // variable-side tail of the second variable block: lanes 0-61 real, 62-63 pad
    for (int r = 0; r < 63; ++r) {
        std::vector<uint32_t> row(64, kPadLane);
        for (int j = 0; j < 62; ++j) row[j] = (uint32_t)(5 * 64 + (j + 1 + r) % 63);
        if (!check_row(row, pool_zero)) { printf("fail vn r %d\n", r); return 1; }
        ++cases;
    }
    // all padding
    {
        std::vector<uint32_t> row(64, kPadLane);
        if (!check_row(row, pool_zero + 3)) { printf("fail all-padding\n"); return 1; }
        ++cases;
    }
    // random rows: random real addresses, random padding subsets, pools at any offset
    std::mt19937 rng(12345);
    for (int t = 0; t < 20000; ++t) {
        std::vector<uint32_t> row(64);
        const int pad_pct = (int)(rng() % 101);
        for (int l = 0; l < 64; ++l) row[l] = (int)(rng() % 100) < pad_pct ? kPadLane : (uint32_t)(rng() % 4096);
        const uint32_t pool = 4096 + (uint32_t)(rng() % 200);
        if (!check_row(row, pool)) { printf("fail random case %d\n", t); return 1; }
        ++cases;
    }
    // several gathers in one table
    {
        std::vector<uint32_t> table(64 * 5, kPadLane);
        for (size_t i = 0; i < table.size(); ++i)
            if (i % 7) table[i] = (uint32_t)(i * 3 % 1000);
        std::vector<uint32_t> placed = table;
        place_padding(placed, 2000);
        for (size_t r = 0; r < table.size(); r += 64) {
            std::vector<uint32_t> b(table.begin() + r, table.begin() + r + 64), a(placed.begin() + r, placed.begin() + r + 64);
            std::vector<uint32_t> a2 = b;
            place_padding(a2, 2000);
            if (a != a2 || !check_row(b, 2000)) { printf("fail table row %zu\n", r / 64); return 1; }
            ++cases;
        }
    }
    printf("ok %d\n", cases);
    return 0;
}
