// Checks the decode launch's frame-to-wave assignment on the host: every
// frame of [0, n) is decoded by exactly one wave, no wave is empty, runs
// never exceed the requested length, and a tapered schedule's runs do not
// grow towards the end of the grid.  The wave-to-frames mapping below is the
// decode kernel's.  Prints "ok <cases>" or the first failing case.
#include <cstdio>
#include <vector>

#include "schedule.h"

using namespace sagms;

static bool check(int64_t n, int fpw, int64_t level_waves, int head) {
    const WaveSchedule s = make_schedule(n, fpw, level_waves, head);
    if (n > 0 && (s.levels < 1 || s.levels > kMaxLevels)) return false;
    if (n == 0) return s.levels == 0;
    std::vector<unsigned char> seen((size_t)n, 0);
    int prev_chunk = 1 << 30;
    for (int k = 0; k < s.levels; ++k) {
        if (s.wave0[k + 1] <= s.wave0[k] || s.frame0[k + 1] <= s.frame0[k]) return false;
        const int lim = fpw > 0 ? fpw : head;
        if (s.chunk[k] < 1 || s.chunk[k] > lim) return false;
        if (fpw == 0 && s.chunk[k] > prev_chunk) return false;
        prev_chunk = s.chunk[k];
    }
    if (s.frame0[0] != 0 || s.frame0[s.levels] != n) return false;
    for (int64_t wave = 0; wave < s.wave0[s.levels]; ++wave) {
        int k = 0;
        while (k + 1 < s.levels && wave >= s.wave0[k + 1]) ++k;
        const int64_t b = s.frame0[k] + (wave - s.wave0[k]) * s.chunk[k];
        const int64_t e = std::min<int64_t>(b + s.chunk[k], s.frame0[k + 1]);
        if (b >= e || b < 0 || e > n) return false;
        for (int64_t f = b; f < e; ++f)
            if (seen[(size_t)f]++) return false;
    }
    for (int64_t f = 0; f < n; ++f)
        if (!seen[(size_t)f]) return false;
    return true;
}

int main() {
    const int64_t ns[] = {0, 1, 2, 3, 7, 8, 9, 63, 64, 65, 1000, 4095, 4096, 4097, 57343, 57344, 57345,
                          65536, 100003, 1 << 20, (1 << 20) + 5};
    const int fpws[] = {0, 1, 2, 3, 8, 16, 1024};
    const int64_t lws[] = {1, 3, 64, 8192, 16384};
    const int heads[] = {1, 2, 8, 16, 32};
    long cases = 0;
    for (int64_t n : ns)
        for (int fpw : fpws)
            for (int64_t lw : lws)
                for (int h : heads) {
                    if (fpw > 0 && (lw != 1 || h != 8)) continue;
                    ++cases;
                    if (!check(n, fpw, lw, h)) {
                        std::printf("FAIL n=%lld fpw=%d level_waves=%lld head=%d\n", (long long)n, fpw,
                                    (long long)lw, h);
                        return 1;
                    }
                }
    std::printf("ok %ld\n", cases);
    return 0;
}
