// Host side of the layered schedule: the layers of a graph (first fit in
// ascending check index: check i joins the first layer none of whose checks
// shares a variable with it, else opens a new one), their passes of at most
// `group` checks, and the host copies of the tables of layered.hip (uploaded
// with the graph's other device tables).
#include <algorithm>

#include "internal.h"

namespace sagms {

namespace {

constexpr int kLayeredMaxLds = 65536;

int round4(int x) { return (x + 3) & ~3; }

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
    size_t widest = 0;
    for (const auto& l : layers) widest = std::max(widest, l.size());
    // lanes per frame: the widest layer, the syndrome and estimate words
    // (one lane each), a power of two up to a whole wavefront
    const size_t need = std::max({widest, (size_t)g->wm, (size_t)g->wn});
    int group = 8;
    while (group < 64 && (size_t)group < need) group *= 2;
    if ((size_t)g->wm > (size_t)group || (size_t)g->wn > (size_t)group)
        return refuse(lh, "layered schedule: code too long");

    lh->pass_check.clear();
    int passes = 0;
    for (const auto& l : layers)
        for (size_t b = 0; b < l.size(); b += group) {
            for (int q = 0; q < group; ++q) lh->pass_check.push_back(b + q < l.size() ? l[b + q] : -1);
            ++passes;
        }
    lh->check_vars.assign((size_t)m * (dc / 2), 0u);
    for (int c = 0; c < m; ++c)
        for (int k = 0; k < dc / 2; ++k)
            lh->check_vars[(size_t)c * (dc / 2) + k] = (uint32_t)(4 * g->cols[g->row_ptr[c] + 2 * k]) |
                                                       ((uint32_t)(4 * g->cols[g->row_ptr[c] + 2 * k + 1]) << 16);
    lh->dc = dc;
    lh->group = group;
    lh->passes = passes;
    lh->npad = round4(n);
    lh->regs = passes <= kLayeredRegPasses;
    // every group of a wavefront updates the same check in the same pass, so
    // its lanes read the same offsets of their own slices.  With the check
    // outputs in LDS, slices 4 words apart modulo the LDS banks keep those
    // reads (and the 4-word reads of a check's compressed outputs) on
    // different banks; with them in registers, the 32 / G groups of a
    // half-wavefront (32 banks) sit G words apart modulo 32.
    if (lh->regs)
        lh->group_words = (lh->npad + 4 * g->wm + 31) / 32 * 32 + (group < 32 ? group : 0);
    else
        lh->group_words = (lh->npad + 4 * m + 4 * g->wm + 63) / 64 * 64 + 4;
    lh->table_words = round4(passes * group + m * (dc / 2) + 2 * (m + 1) + n + 2 * g->wm);
    const int frames = 64 / group;
    if ((size_t)(lh->table_words + frames * lh->group_words) * 4 > (size_t)kLayeredMaxLds)
        return refuse(lh, "layered schedule: code too large for one wavefront's LDS");
    lh->status = SAGMS_OK;
    lh->why.clear();
    return SAGMS_OK;
}

void plan_layers(Graph* g) { (void)plan(g, &g->layered); }

}  // namespace sagms
