// Frame-to-wave assignment of a decode launch (host code, no HIP types).
// The launch's waves are cut into levels: wave w of level k (waves
// [wave0[k], wave0[k+1])) decodes chunk[k] consecutive frames starting at
// frame0[k] + (w - wave0[k]) chunk[k] and ending no later than frame0[k+1].
// Every frame of [0, n) belongs to exactly one wave.
#pragma once

#include <algorithm>
#include <cstdint>

namespace sagms {

constexpr int kMaxLevels = 8;
struct WaveSchedule {
    int64_t wave0[kMaxLevels + 1];
    int64_t frame0[kMaxLevels + 1];
    int32_t chunk[kMaxLevels];
    int32_t levels;
};

// One level of `chunk` frames per wave over frames [f0, f1).
inline void add_level(WaveSchedule& s, int64_t f0, int64_t f1, int chunk) {
    if (f1 <= f0) return;
    const int k = s.levels++;
    s.frame0[k] = f0;
    s.chunk[k] = chunk;
    s.wave0[k + 1] = s.wave0[k] + (f1 - f0 + chunk - 1) / chunk;
    s.frame0[k + 1] = f1;
}

// Uniform (fpw > 0): chunks of fpw frames.  Tapered (fpw = 0): counted from
// the end of the launch, level_waves waves of 1 frame, then level_waves
// waves of 2, 4, ... up to head / 2 frames, and every frame before those in
// chunks of head frames.  With level_waves = the waves resident on the
// device at once, the waves dispatched last hold the fewest frames.
inline WaveSchedule make_schedule(int64_t n, int fpw, int64_t level_waves, int head) {
    WaveSchedule s{};
    if (fpw > 0) {
        add_level(s, 0, n, fpw);
        return s;
    }
    int64_t tail[kMaxLevels] = {};
    int chunks[kMaxLevels] = {};
    int nt = 0;
    int64_t left = n;
    for (int c = 1; c < head && nt < kMaxLevels - 1; c *= 2) {
        const int64_t take = std::min<int64_t>(left, level_waves * c);
        chunks[nt] = c;
        tail[nt++] = take;
        left -= take;
    }
    add_level(s, 0, left, head);
    int64_t f = left;
    for (int i = nt - 1; i >= 0; --i) {
        add_level(s, f, f + tail[i], chunks[i]);
        f += tail[i];
    }
    return s;
}

}  // namespace sagms
