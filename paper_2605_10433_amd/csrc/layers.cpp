// Host side of the layered schedule: the layers of a graph (first fit in
// ascending check index: check i joins the first layer none of whose checks
// shares a variable with it, else opens a new one), the passes of at most
// `group` checks that run them, and the host copies of the tables of
// layered.hip (uploaded with the graph's other device tables).
#include <algorithm>

#include "internal.h"
#include "lane_code.h"

namespace sagms {

namespace {

constexpr int kLayeredMaxLds = 65536;
// time of a pass with the check outputs in LDS over one with them in
// registers (same schedule, l = 63 workload)
constexpr double kLdsFormCost = 1.18;
constexpr int kLdsPerCu = 163840;  // bytes of LDS per compute unit

int round4(int x) { return (x + 3) & ~3; }

// True when g's rows are those compiled into the one-lane kernel (as sets:
// the order of a row's variables does not change any result).
bool is_lane_code(const Graph* g) {
    if (g->m != lane::kL || g->n != lane::kN) return false;
    for (int c = 0; c < lane::kL; ++c) {
        if (g->row_ptr[c + 1] - g->row_ptr[c] != lane::kDC) return false;
        std::vector<int> mine(g->cols.begin() + g->row_ptr[c], g->cols.begin() + g->row_ptr[c + 1]);
        std::vector<int> want(lane::kRows.var[c], lane::kRows.var[c] + lane::kDC);
        std::sort(mine.begin(), mine.end());
        std::sort(want.begin(), want.end());
        if (mine != want) return false;
    }
    return true;
}

// LDS words of one frame's slice.  Every group of a wavefront updates the
// same check in the same pass, so its lanes read the same offsets of their
// own slices.  With the check outputs in LDS, slices 4 words apart modulo the
// LDS banks keep those reads (and the 4-word reads of a check's compressed
// outputs) on different banks; with them in registers, the 32 / G groups of
// a half-wavefront (32 banks) sit G words apart modulo 32.
int group_words(int n, int m, int wm, int group, bool regs) {
    const int npad = round4(n);
    if (regs) return (npad + 4 * wm + 31) / 32 * 32 + (group < 32 ? group : 0);
    return (npad + 4 * m + 4 * wm + 63) / 64 * 64 + 4;
}

// LDS words of the tables in front of the slices: pass table, variable
// pairs, gain pairs, prior, residual bits of the prior's hard decision.
int table_words(int passes, int group, int m, int dc, int n, int wm) {
    return round4(passes * group + m * (dc / 2) + 2 * (m + 1) + n + 2 * wm);
}

}  // namespace

static int refuse(LayeredHost* lh, const char* why) {
    lh->status = SAGMS_EUNSUPPORTED;
    lh->why = why;
    return lh->status;
}

static int plan(const Graph* g, LayeredHost* lh) {
    if (g->joint) return refuse(lh, "layered schedule: joint graphs decode with the flooding schedule");
    const int m = g->m, n = g->n;
    const int dc = g->row_ptr[1] - g->row_ptr[0];
    for (int c = 0; c < m; ++c)
        if (g->row_ptr[c + 1] - g->row_ptr[c] != dc)
            return refuse(lh, "layered schedule: needs every check of the same degree");
    if (dc != 6 && dc != 8 && dc != 10) return refuse(lh, "layered schedule: check degree not compiled (6, 8 or 10)");
    if (!g->shape_ok) return refuse(lh, "layered schedule: no decode kernel fits the graph");
    // variables are held as 16-bit byte offsets (4 j)
    if (n > 0x3FFF) return refuse(lh, "layered schedule: n must be < 16384");

    // first-fit layers
    std::vector<std::vector<int>> layers;
    std::vector<std::vector<char>> used;
    for (int c = 0; c < m; ++c) {
        size_t l = 0;
        for (; l < layers.size(); ++l) {
            bool clash = false;
            for (int e = g->row_ptr[c]; e < g->row_ptr[c + 1] && !clash; ++e) clash = used[l][g->cols[e]] != 0;
            if (!clash) break;
        }
        if (l == layers.size()) {
            layers.emplace_back();
            used.emplace_back(n, 0);
        }
        layers[l].push_back(c);
        for (int e = g->row_ptr[c]; e < g->row_ptr[c + 1]; ++e) used[l][g->cols[e]] = 1;
    }
    // Passes for each lane-group size G: the checks in (layer, position)
    // order, each in the earliest pass that follows every pass holding a
    // check with a variable in common and that has a free lane.  Every
    // variable then meets its checks in layer order, as in the layer-by-layer
    // schedule, so the results are the same; a pass may hold checks of
    // several layers.  G is chosen by the lane slots per frame and round,
    // passes x G, with the LDS form of the outputs weighted by its measured
    // extra cost and plans with fewer than 8 resident wavefronts per CU by
    // the missing ones; on a tie the larger G (the shorter pass chain).
    // The compiled l = 63 code: one lane per frame updates the checks one
    // after another in (layer, position) order, the order of these layers.
    if (is_lane_code(g)) {
        std::vector<int32_t> order;
        for (const auto& l : layers) order.insert(order.end(), l.begin(), l.end());
        if (std::equal(order.begin(), order.end(), lane::kOrder.check) && (int)layers.size() == lane::kOrder.layers) {
            lh->group = 1;
            lh->passes = m;
            lh->regs = true;
            lh->group_words = 0;
            lh->table_words = 0;
            lh->pass_check = order;
            lh->check_vars.assign((size_t)m * (dc / 2), 0u);  // not read by the kernel; kept for the upload
            lh->dc = dc;
            lh->npad = round4(n);
            lh->status = SAGMS_OK;
            lh->why.clear();
            return SAGMS_OK;
        }
    }
    const int wm = g->wm, wn = g->wn;
    if (wm > 64 || wn > 64) return refuse(lh, "layered schedule: code too long");
    std::vector<int> last(n);
    double best_cost = 0.0;
    int best_group = 0;
    for (int group = 8; group <= 64; group *= 2) {
        // lanes per frame: the syndrome and estimate words need one lane each
        if (group < wm || group < wn) continue;
        std::vector<int> fill;  // checks per pass
        std::vector<int> where(m);
        std::fill(last.begin(), last.end(), -1);
        for (const auto& l : layers)
            for (int c : l) {
                int p = 0;
                for (int e = g->row_ptr[c]; e < g->row_ptr[c + 1]; ++e) p = std::max(p, last[g->cols[e]] + 1);
                while (p < (int)fill.size() && fill[p] == group) ++p;
                if (p == (int)fill.size()) fill.push_back(0);
                ++fill[p];
                where[c] = p;
                for (int e = g->row_ptr[c]; e < g->row_ptr[c + 1]; ++e) last[g->cols[e]] = p;
            }
        const int passes = (int)fill.size();
        const bool regs = passes <= kLayeredRegPasses;
        const int gw = group_words(n, m, wm, group, regs);
        const int tw = table_words(passes, group, m, dc, n, wm);
        const int lds = (tw + (64 / group) * gw) * 4;
        if (lds > kLayeredMaxLds) continue;
        // resident wavefronts per CU (registers: 3 per SIMD in the register
        // form, 6 in the LDS form; LDS); below 8 a pass's LDS latency shows
        const int waves = std::min(regs ? 12 : 24, kLdsPerCu / lds);
        const double cost = (double)passes * group * (regs ? 1.0 : kLdsFormCost) * std::max(1.0, 8.0 / waves);
        if (best_group && cost > best_cost) continue;
        best_cost = cost;
        best_group = group;
        lh->passes = passes;
        lh->regs = regs;
        lh->group_words = gw;
        lh->table_words = tw;
        // lanes of a pass in (layer, position) order of their checks
        lh->pass_check.assign((size_t)passes * group, -1);
        std::vector<int> lanes(passes, 0);
        for (const auto& l : layers)
            for (int c : l) lh->pass_check[(size_t)where[c] * group + lanes[where[c]]++] = c;
    }
    if (!best_group) return refuse(lh, "layered schedule: code too large for one wavefront's LDS");
    lh->check_vars.assign((size_t)m * (dc / 2), 0u);
    for (int c = 0; c < m; ++c)
        for (int k = 0; k < dc / 2; ++k)
            lh->check_vars[(size_t)c * (dc / 2) + k] = (uint32_t)(4 * g->cols[g->row_ptr[c] + 2 * k]) |
                                                       ((uint32_t)(4 * g->cols[g->row_ptr[c] + 2 * k + 1]) << 16);
    lh->dc = dc;
    lh->group = best_group;
    lh->npad = round4(n);
    lh->status = SAGMS_OK;
    lh->why.clear();
    return SAGMS_OK;
}

void plan_layers(Graph* g) { (void)plan(g, &g->layered); }

}  // namespace sagms
