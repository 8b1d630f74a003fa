#pragma once
// Placement of the padding lanes of the decoder's LDS gathers (host side).
//
// The LDS serves a wavefront's 64 lanes as two halves of 32, each against
// 32 banks of 4 bytes: lanes 0-31 and 32-63 on the same banks cost nothing,
// while two different words of one bank within a half cost an extra cycle
// (measured on gfx950).  Lanes that read the same word get it broadcast.
#include <cstddef>
#include <cstdint>
#include <vector>

namespace sagms {

constexpr int kLdsBanks = 32;
constexpr uint32_t kPadLane = 0xFFFFFFFFu;  // table entry of a padding lane before placement

// `table` holds 64-lane gathers (rows of 64 LDS word indices); padding lanes
// are kPadLane.  Points the padding lanes of each half of each gather at one
// word of the 64-word pool starting at `pool` (all holding the padding
// value): the word in the bank that the real lanes of that half use least,
// so a bank none of them uses when there is one.
inline void place_padding(std::vector<uint32_t>& table, uint32_t pool) {
    for (size_t half = 0; half + 32 <= table.size(); half += 32) {
        int load[kLdsBanks] = {};
        for (int l = 0; l < 32; ++l)
            if (table[half + l] != kPadLane) ++load[table[half + l] % kLdsBanks];
        int best = 0;
        for (int b = 1; b < kLdsBanks; ++b)
            if (load[b] < load[best]) best = b;
        const uint32_t word = pool + (uint32_t)((best - (int)(pool % kLdsBanks) + kLdsBanks) % kLdsBanks);
        for (int l = 0; l < 32; ++l)
            if (table[half + l] == kPadLane) table[half + l] = word;
    }
}

}  // namespace sagms
