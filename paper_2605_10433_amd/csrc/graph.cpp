// Host side of libsagms: Tanner graphs, GF(2) algebra for the logical
// judge, per-device tables, error reporting and the graph entry points.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "internal.h"
#include "lds_pad.h"

namespace sagms {

static thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(SAGMS_EHIP, "%s failed: %s", what, hipGetErrorString(e));
}

// ---- GF(2) elimination on packed rows ----------------------------------
static inline bool bit(const uint64_t* row, int j) { return (row[j >> 6] >> (j & 63)) & 1u; }

// Reduces `rows` (nrows x wn words) in place to row-echelon form; returns the
// rank and the pivot column of each of the first `rank` rows.
static int gf2_echelon(std::vector<uint64_t>& rows, int nrows, int wn, int ncols, std::vector<int>* pivots) {
    int r = 0;
    for (int c = 0; c < ncols && r < nrows; ++c) {
        int p = -1;
        for (int i = r; i < nrows; ++i)
            if (bit(&rows[(size_t)i * wn], c)) { p = i; break; }
        if (p < 0) continue;
        if (p != r)
            for (int w = 0; w < wn; ++w) std::swap(rows[(size_t)p * wn + w], rows[(size_t)r * wn + w]);
        for (int i = 0; i < nrows; ++i)
            if (i != r && bit(&rows[(size_t)i * wn], c))
                for (int w = 0; w < wn; ++w) rows[(size_t)i * wn + w] ^= rows[(size_t)r * wn + w];
        if (pivots) pivots->push_back(c);
        ++r;
    }
    return r;
}

int gf2_rank(std::vector<uint64_t> rows, int nrows, int wn) {
    return gf2_echelon(rows, nrows, wn, wn * 64, nullptr);
}

// Basis of {x : A x = 0} for A given as packed rows.
static std::vector<uint64_t> gf2_kernel(std::vector<uint64_t> a, int nrows, int wn, int ncols, int* dim) {
    std::vector<int> piv;
    int r = gf2_echelon(a, nrows, wn, ncols, &piv);
    std::vector<char> is_piv(ncols, 0);
    for (int c : piv) is_piv[c] = 1;
    std::vector<uint64_t> out;
    int d = 0;
    for (int f = 0; f < ncols; ++f) {
        if (is_piv[f]) continue;
        std::vector<uint64_t> v(wn, 0);
        v[f >> 6] |= 1ull << (f & 63);
        for (int i = 0; i < r; ++i)
            if (bit(&a[(size_t)i * wn], f)) v[piv[i] >> 6] |= 1ull << (piv[i] & 63);
        out.insert(out.end(), v.begin(), v.end());
        ++d;
    }
    *dim = d;
    return out;
}

// ---- decode shapes and LDS layout ----------------------------------------
static const DecodeShape kShapes[] = {
#define SAGMS_SHAPE_ENTRY(I, DC, DV, CPL, VPL) {DC, DV, CPL, VPL},
    SAGMS_DECODE_SHAPES(SAGMS_SHAPE_ENTRY)
#undef SAGMS_SHAPE_ENTRY
};
static_assert(sizeof(kShapes) / sizeof(kShapes[0]) == kNumShapes, "shape list");

int shape_index(const DecodeShape& s) {
    for (int i = 0; i < kNumShapes; ++i)
        if (kShapes[i].dc == s.dc && kShapes[i].dv == s.dv && kShapes[i].cpl == s.cpl && kShapes[i].vpl == s.vpl)
            return i;
    return -1;
}

bool pick_shape(int m, int n, int dc, int dv, DecodeShape* out) {
    bool found = false;
    int best = 0;
    for (const DecodeShape& s : kShapes) {
        if (s.dc < dc || s.dv < dv || 64 * s.cpl < m || 64 * s.vpl < n) continue;
        int cost = s.cpl * s.dc * 3 + s.vpl * s.dv;  // registers held per lane, roughly
        if (!found || cost < best) { *out = s; best = cost; found = true; }
    }
    return found;
}

DecodeLayout make_layout(const DecodeShape& s) {
    DecodeLayout L;
    L.cw = 64 * s.cpl;
    L.zero = s.dc * L.cw;
    L.post0 = L.zero + 64;
    L.padpost = L.post0 + 64 * s.vpl;
    L.gain0 = L.padpost + 64;  // 8-byte aligned pairs
    L.words = L.gain0 + 2 * (L.cw + 1);
    return L;
}

static const DecodeShape kJointShapes[] = {
#define SAGMS_JOINT_ENTRY(I, DC, DV, CPL, VPL) {DC, DV, CPL, VPL},
    SAGMS_JOINT_SHAPES(SAGMS_JOINT_ENTRY)
#undef SAGMS_JOINT_ENTRY
};
static_assert(sizeof(kJointShapes) / sizeof(kJointShapes[0]) == kNumJointShapes, "joint shape list");

bool pick_joint_shape(int m, int n, int dc, int dvh, DecodeShape* out) {
    bool found = false;
    int best = 0;
    for (const DecodeShape& s : kJointShapes) {
        if (s.dc < dc || s.dv < 2 * dvh || 64 * s.cpl < m || 64 * s.vpl < n) continue;
        int cost = s.cpl * s.dc * 3 + s.vpl * s.dv;
        if (!found || cost < best) { *out = s; best = cost; found = true; }
    }
    return found;
}

JointLayout make_joint_layout(const DecodeShape& s) {
    JointLayout L;
    L.cw = 64 * s.cpl;
    L.zero = s.dc * L.cw;
    L.pairx = L.zero + 64;
    L.pairz = L.pairx + 128 * s.vpl;
    L.padpair = L.pairz + 128 * s.vpl;
    L.gain0 = L.padpair + 128;
    L.words = L.gain0 + 2 * (L.cw + 1);
    return L;
}

// Builds the per-lane LDS address tables for the chosen shape.
static void build_lane_tables(Graph* g) {
    const DecodeShape& s = g->shape;
    const DecodeLayout& L = g->layout;
    g->cn_addr_host.assign((size_t)s.cpl * s.dc * 64, kPadLane);
    g->vn_addr_host.assign((size_t)s.vpl * s.dv * 64, kPadLane);
    for (int c = 0; c < g->m; ++c)
        for (int p = 0; p < g->row_ptr[c + 1] - g->row_ptr[c]; ++p) {
            int j = g->cols[g->row_ptr[c] + p];
            g->cn_addr_host[((size_t)(c / 64) * s.dc + p) * 64 + (c % 64)] = (uint32_t)(L.post0 + j);
        }
    for (int j = 0; j < g->n; ++j)
        for (size_t r = 0; r < g->var_edges[j].size(); ++r) {
            int c = g->var_edges[j][r].first, p = g->var_edges[j][r].second;
            g->vn_addr_host[((size_t)(j / 64) * s.dv + r) * 64 + (j % 64)] = (uint32_t)(p * L.cw + c);
        }
    place_padding(g->cn_addr_host, (uint32_t)L.padpost);
    place_padding(g->vn_addr_host, (uint32_t)L.zero);
}

// Every variable's (check, position) pairs in posterior-sum order: ascending
// check index, or for a GB code the order of the polynomial terms (variable
// i of the first block meets check (i + b_t) mod l at position t, variable
// l + i of the second block check (i + a_t) mod l at position wb + t).
static void build_var_edges(Graph* g) {
    g->var_edges.assign(g->n, {});
    if (g->is_gb) {
        const int l = g->gb_l, wb = (int)g->gb_b.size();
        for (int i = 0; i < l; ++i) {
            for (int t = 0; t < wb; ++t) g->var_edges[i].push_back({(i + g->gb_b[t]) % l, t});
            for (int t = 0; t < (int)g->gb_a.size(); ++t) g->var_edges[l + i].push_back({(i + g->gb_a[t]) % l, wb + t});
        }
        return;
    }
    for (int c = 0; c < g->m; ++c)
        for (int p = 0; p < g->row_ptr[c + 1] - g->row_ptr[c]; ++p) g->var_edges[g->cols[g->row_ptr[c] + p]].push_back({c, p});
    for (auto& v : g->var_edges) std::sort(v.begin(), v.end());
}

// ---- graph construction ------------------------------------------------
static int finish_graph(Graph* g, const std::vector<int>& row_ptr_o, const std::vector<int>& cols_o, int m_other) {
    g->E = g->row_ptr[g->m];
    g->wn = (g->n + 63) / 64;
    g->wm = (g->m + 63) / 64;
    g->we = g->wn;
    g->rows_bits.assign((size_t)g->m * g->wn, 0);
    std::vector<int> vdeg(g->n, 0);
    g->dc_max = 0;
    for (int c = 0; c < g->m; ++c) {
        int d = g->row_ptr[c + 1] - g->row_ptr[c];
        g->dc_max = std::max(g->dc_max, d);
        for (int t = g->row_ptr[c]; t < g->row_ptr[c + 1]; ++t) {
            int j = g->cols[t];
            g->rows_bits[(size_t)c * g->wn + (j >> 6)] |= 1ull << (j & 63);
            vdeg[j]++;
        }
    }
    g->dv_max = g->n ? *std::max_element(vdeg.begin(), vdeg.end()) : 0;
    g->have_other = m_other > 0;
    if (g->have_other) {
        std::vector<uint64_t> other((size_t)m_other * g->wn, 0);
        for (int c = 0; c < m_other; ++c)
            for (int t = row_ptr_o[c]; t < row_ptr_o[c + 1]; ++t)
                other[(size_t)c * g->wn + (cols_o[t] >> 6)] |= 1ull << (cols_o[t] & 63);
        // CSS condition: every row of H is orthogonal to every row of H_other
        for (int a = 0; a < g->m; ++a)
            for (int b = 0; b < m_other; ++b) {
                int par = 0;
                for (int w = 0; w < g->wn; ++w)
                    par ^= __builtin_popcountll(g->rows_bits[(size_t)a * g->wn + w] & other[(size_t)b * g->wn + w]) & 1;
                if (par) return fail(SAGMS_EINVAL, "row %d of H and row %d of H_other anticommute", a, b);
            }
        // logical basis: ker(H_other) modulo rowspace(H)
        int kdim = 0;
        std::vector<uint64_t> kern = gf2_kernel(other, m_other, g->wn, g->n, &kdim);
        std::vector<uint64_t> acc = g->rows_bits;
        int acc_rows = g->m;
        int acc_rank = gf2_rank(acc, acc_rows, g->wn);
        g->logicals.clear();
        for (int t = 0; t < kdim; ++t) {
            std::vector<uint64_t> trial = acc;
            trial.insert(trial.end(), kern.begin() + (size_t)t * g->wn, kern.begin() + (size_t)(t + 1) * g->wn);
            int r = gf2_rank(trial, acc_rows + 1, g->wn);
            if (r > acc_rank) {
                acc.swap(trial);
                acc_rows++;
                acc_rank = r;
                g->logicals.insert(g->logicals.end(), kern.begin() + (size_t)t * g->wn,
                                   kern.begin() + (size_t)(t + 1) * g->wn);
            }
        }
        g->k = (int)(g->logicals.size() / g->wn);
    }
    build_var_edges(g);
    g->shape_ok = pick_shape(g->m, g->n, g->dc_max, g->dv_max, &g->shape);
    if (g->shape_ok) {
        g->layout = make_layout(g->shape);
        build_lane_tables(g);
    }
    return SAGMS_OK;
}

// Basis of ker(a) modulo rowspace(b) (a, b: packed rows over ncols bits).
static std::vector<uint64_t> logical_rows(const std::vector<uint64_t>& a, int ma, const std::vector<uint64_t>& b,
                                          int mb, int wn, int ncols) {
    int kdim = 0;
    std::vector<uint64_t> kern = gf2_kernel(a, ma, wn, ncols, &kdim);
    std::vector<uint64_t> acc = b, out;
    int acc_rows = mb, acc_rank = gf2_rank(acc, acc_rows, wn);
    for (int t = 0; t < kdim; ++t) {
        std::vector<uint64_t> trial = acc;
        trial.insert(trial.end(), kern.begin() + (size_t)t * wn, kern.begin() + (size_t)(t + 1) * wn);
        const int r = gf2_rank(trial, acc_rows + 1, wn);
        if (r > acc_rank) {
            acc.swap(trial);
            acc_rows++;
            acc_rank = r;
            out.insert(out.end(), kern.begin() + (size_t)t * wn, kern.begin() + (size_t)(t + 1) * wn);
        }
    }
    return out;
}

// Joint graph of a GB code (set up by sagms_build_gb_joint): rows over the
// (x | z) planes, logical rows, each variable's X-type then Z-type checks in
// posterior-sum order, shape, layout and lane tables of the joint kernel.
static int finish_joint(Graph* g) {
    const int l = g->gb_l, n = g->n, m = g->m;
    g->E = g->row_ptr[m];
    g->wn = (n + 63) / 64;
    g->wm = (m + 63) / 64;
    g->we = 2 * g->wn;
    const int wn = g->wn;
    g->rows_bits.assign((size_t)m * g->we, 0);
    std::vector<uint64_t> hx((size_t)l * wn, 0), hz((size_t)l * wn, 0);
    std::vector<int> vdeg(n, 0);
    g->dc_max = 0;
    for (int c = 0; c < m; ++c) {
        const bool xtype = c < l;
        g->dc_max = std::max(g->dc_max, g->row_ptr[c + 1] - g->row_ptr[c]);
        for (int t = g->row_ptr[c]; t < g->row_ptr[c + 1]; ++t) {
            const int j = g->cols[t];
            // an X-type check sees the Z part of an error, a Z-type check the X part
            g->rows_bits[(size_t)c * g->we + (xtype ? wn : 0) + (j >> 6)] |= 1ull << (j & 63);
            (xtype ? hx : hz)[(size_t)(xtype ? c : c - l) * wn + (j >> 6)] |= 1ull << (j & 63);
            vdeg[j]++;
        }
    }
    g->dv_max = *std::max_element(vdeg.begin(), vdeg.end());
    for (int a = 0; a < l; ++a)
        for (int b = 0; b < l; ++b) {
            int par = 0;
            for (int w = 0; w < wn; ++w) par ^= __builtin_popcountll(hx[(size_t)a * wn + w] & hz[(size_t)b * wn + w]) & 1;
            if (par) return fail(SAGMS_EINVAL, "X-type row %d and Z-type row %d anticommute", a, b);
        }
    // Z-type logicals ker(H_X) mod rowspace(H_Z) act on the X part of a
    // residual, X-type logicals ker(H_Z) mod rowspace(H_X) on its Z part
    const std::vector<uint64_t> zl = logical_rows(hx, l, hz, l, wn, n), xl = logical_rows(hz, l, hx, l, wn, n);
    g->k = (int)(zl.size() / wn);
    if ((int)(xl.size() / wn) != g->k) return fail(SAGMS_EINVAL, "logical dimensions differ (internal)");
    g->logicals.assign((size_t)2 * g->k * g->we, 0);
    for (int t = 0; t < g->k; ++t)
        for (int w = 0; w < wn; ++w) {
            g->logicals[(size_t)t * g->we + w] = zl[(size_t)t * wn + w];
            g->logicals[(size_t)(g->k + t) * g->we + wn + w] = xl[(size_t)t * wn + w];
        }
    g->have_other = true;
    // posterior-sum order: variable i < l meets X-type checks (i - a_t) mod l
    // and Z-type checks l + (i + b_t) mod l; variable l + i the X-type checks
    // (i - b_t) mod l and Z-type checks l + (i + a_t) mod l, in term order
    auto position = [&](int c, int j) {
        for (int t = g->row_ptr[c]; t < g->row_ptr[c + 1]; ++t)
            if (g->cols[t] == j) return t - g->row_ptr[c];
        return -1;
    };
    const std::vector<int>&A = g->gb_a, &B = g->gb_b;
    std::vector<std::vector<int>> xc(n), zc(n);
    for (int i = 0; i < l; ++i) {
        for (int a : A) xc[i].push_back(((i - a) % l + l) % l);
        for (int b : B) zc[i].push_back(l + (i + b) % l);
        for (int b : B) xc[l + i].push_back(((i - b) % l + l) % l);
        for (int a : A) zc[l + i].push_back(l + (i + a) % l);
    }
    g->dvh = 0;
    for (int j = 0; j < n; ++j) g->dvh = std::max({g->dvh, (int)xc[j].size(), (int)zc[j].size()});
    g->var_edges.assign(n, {});
    for (int j = 0; j < n; ++j) {
        for (int c : xc[j]) g->var_edges[j].push_back({c, position(c, j)});
        for (int c : zc[j]) g->var_edges[j].push_back({c, position(c, j)});
        for (const auto& e : g->var_edges[j])
            if (e.second < 0) return fail(SAGMS_EINVAL, "joint graph: variable %d missing from check %d (internal)", j, e.first);
    }
    g->shape_ok = pick_joint_shape(m, n, g->dc_max, g->dvh, &g->shape);
    if (!g->shape_ok) return SAGMS_OK;
    const DecodeShape& s = g->shape;
    const JointLayout& L = g->jlayout = make_joint_layout(s);
    g->cn_addr_host.assign((size_t)s.cpl * s.dc * 64, kPadLane);
    g->vn_addr_host.assign((size_t)s.vpl * s.dv * 64, kPadLane);
    for (int c = 0; c < m; ++c)
        for (int p = 0; p < g->row_ptr[c + 1] - g->row_ptr[c]; ++p) {
            const int j = g->cols[g->row_ptr[c] + p];
            g->cn_addr_host[((size_t)(c / 64) * s.dc + p) * 64 + (c % 64)] = (uint32_t)((c < l ? L.pairx : L.pairz) + 2 * j);
        }
    const int dvh = s.dv / 2;
    for (int j = 0; j < n; ++j) {
        for (size_t r = 0; r < xc[j].size(); ++r) {
            const auto& e = g->var_edges[j][r];
            g->vn_addr_host[((size_t)(j / 64) * s.dv + r) * 64 + (j % 64)] = (uint32_t)(e.second * L.cw + e.first);
        }
        for (size_t r = 0; r < zc[j].size(); ++r) {
            const auto& e = g->var_edges[j][xc[j].size() + r];
            g->vn_addr_host[((size_t)(j / 64) * s.dv + dvh + r) * 64 + (j % 64)] = (uint32_t)(e.second * L.cw + e.first);
        }
    }
    // padding: checks read the (+inf, +0) pair at padpair (a broadcast),
    // variables a zero word of the pool
    for (uint32_t& v : g->cn_addr_host)
        if (v == kPadLane) v = (uint32_t)L.padpair;
    place_padding(g->vn_addr_host, (uint32_t)L.zero);
    return SAGMS_OK;
}

static int check_csr(int32_t m, int32_t n, const int32_t* rp, const int32_t* ci, const char* name, bool need_deg2) {
    if (!rp || !ci) return fail(SAGMS_EINVAL, "%s: null CSR pointer", name);
    if (rp[0] != 0) return fail(SAGMS_EINVAL, "%s: row_ptr[0] must be 0", name);
    std::vector<char> seen(n, 0);
    for (int i = 0; i < m; ++i) {
        if (rp[i + 1] < rp[i]) return fail(SAGMS_EINVAL, "%s: row_ptr decreases at row %d", name, i);
        if (need_deg2 && rp[i + 1] - rp[i] < 2)
            return fail(SAGMS_EINVAL, "%s: check %d has degree %d (< 2)", name, i, rp[i + 1] - rp[i]);
        for (int t = rp[i]; t < rp[i + 1]; ++t) {
            int j = ci[t];
            if (j < 0 || j >= n) return fail(SAGMS_EINVAL, "%s: column %d out of range in row %d", name, j, i);
            if (seen[j]) return fail(SAGMS_EINVAL, "%s: column %d repeated in row %d", name, j, i);
            seen[j] = 1;
        }
        for (int t = rp[i]; t < rp[i + 1]; ++t) seen[ci[t]] = 0;
    }
    return SAGMS_OK;
}

static int publish(Graph* g, sagms_graph* out);

static int build(int32_t m, int32_t n, const std::vector<int>& rp, const std::vector<int>& ci, int32_t m_other,
                 const std::vector<int>& rpo, const std::vector<int>& cio, sagms_graph* out,
                 const std::vector<int>* gb_a = nullptr, const std::vector<int>* gb_b = nullptr) {
    Graph* g = new (std::nothrow) Graph();
    if (!g) return fail(SAGMS_ENOMEM, "graph allocation failed");
    g->m = m;
    g->n = n;
    if (gb_a && gb_b) {
        g->is_gb = true;
        g->gb_l = m;
        g->gb_a = *gb_a;
        g->gb_b = *gb_b;
    }
    g->row_ptr = rp;
    g->cols = ci;
    int rc = finish_graph(g, rpo, cio, m_other);
    if (rc != SAGMS_OK) {
        delete g;
        return rc;
    }
    return publish(g, out);
}

// Plans the layered schedule, copies the tables to the current device if the
// process has one (host-only use needs none: the device calls then report a
// graph without tables) and hands the graph out.
static int publish(Graph* g, sagms_graph* out) {
    plan_layers(g);
    int rc = SAGMS_OK;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
        DeviceTables* t = nullptr;
        rc = upload_tables(g, &t);
        if (rc != SAGMS_OK) {
            const std::string why = g_last_error;
            (void)sagms_destroy_graph(reinterpret_cast<sagms_graph>(g));
            g_last_error = why;
            return rc;
        }
    } else {
        (void)hipGetLastError();
    }
    *out = reinterpret_cast<sagms_graph>(g);
    return SAGMS_OK;
}

// ---- per-device tables ------------------------------------------------
static int upload_locked(Graph* g, DeviceTables* t) {
    size_t ncols = (size_t)g->m * std::max(g->dc_max, 1);
    std::vector<int32_t> cols(ncols, -1);
    for (int c = 0; c < g->m; ++c)
        for (int p = 0; p < g->row_ptr[c + 1] - g->row_ptr[c]; ++p)  // joint X-type rows read the Z plane
            cols[(size_t)c * std::max(g->dc_max, 1) + p] = g->cols[g->row_ptr[c] + p] + (g->joint && c < g->m / 2 ? g->n : 0);
    SAGMS_HIP(hipMalloc(&t->cols, std::max<size_t>(ncols, 1) * sizeof(int32_t)));
    SAGMS_HIP(hipMemcpy(t->cols, cols.data(), ncols * sizeof(int32_t), hipMemcpyHostToDevice));
    SAGMS_HIP(hipMalloc(&t->rows, g->rows_bits.size() * sizeof(uint64_t)));
    SAGMS_HIP(hipMemcpy(t->rows, g->rows_bits.data(), g->rows_bits.size() * sizeof(uint64_t), hipMemcpyHostToDevice));
    if (g->shape_ok) {
        SAGMS_HIP(hipMalloc(&t->cn_addr, g->cn_addr_host.size() * sizeof(uint32_t)));
        SAGMS_HIP(hipMemcpy(t->cn_addr, g->cn_addr_host.data(), g->cn_addr_host.size() * sizeof(uint32_t),
                            hipMemcpyHostToDevice));
        SAGMS_HIP(hipMalloc(&t->vn_addr, g->vn_addr_host.size() * sizeof(uint32_t)));
        SAGMS_HIP(hipMemcpy(t->vn_addr, g->vn_addr_host.data(), g->vn_addr_host.size() * sizeof(uint32_t),
                            hipMemcpyHostToDevice));
    }
    if (g->k > 0) {
        SAGMS_HIP(hipMalloc(&t->logicals, g->logicals.size() * sizeof(uint64_t)));
        SAGMS_HIP(hipMemcpy(t->logicals, g->logicals.data(), g->logicals.size() * sizeof(uint64_t),
                            hipMemcpyHostToDevice));
    }
    const LayeredHost& lh = g->layered;
    if (lh.status == SAGMS_OK) {
        LayeredPlan& lp = t->layered;
        lp.dc = lh.dc;
        lp.group = lh.group;
        lp.passes = lh.passes;
        lp.npad = lh.npad;
        lp.group_words = lh.group_words;
        lp.table_words = lh.table_words;
        lp.regs = lh.regs;
        SAGMS_HIP(hipMalloc(&lp.pass_check, lh.pass_check.size() * sizeof(int32_t)));
        SAGMS_HIP(hipMemcpy(lp.pass_check, lh.pass_check.data(), lh.pass_check.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice));
        SAGMS_HIP(hipMalloc(&lp.check_vars, lh.check_vars.size() * sizeof(uint32_t)));
        SAGMS_HIP(hipMemcpy(lp.check_vars, lh.check_vars.data(), lh.check_vars.size() * sizeof(uint32_t),
                            hipMemcpyHostToDevice));
    }
    return SAGMS_OK;
}

static void free_tables(DeviceTables* t) {
    (void)hipFree(t->cols);
    (void)hipFree(t->rows);
    (void)hipFree(t->cn_addr);
    (void)hipFree(t->vn_addr);
    (void)hipFree(t->logicals);
    (void)hipFree(t->layered.pass_check);
    (void)hipFree(t->layered.check_vars);
    *t = DeviceTables{};
}

int upload_tables(Graph* g, DeviceTables** out) {
    int dev = 0;
    SAGMS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SAGMS_EUNSUPPORTED, "device index %d too large", dev);
    std::lock_guard<std::mutex> lock(g->mu);
    DeviceTables* t = &g->dev[dev];
    if (!t->ready) {
        int rc = scratch_setup();  // the device's queue counters for sagms_decode_segments
        if (rc) return rc;
        rc = upload_locked(g, t);
        if (rc) {
            free_tables(t);
            return rc;
        }
        t->ready = true;
    }
    *out = t;
    return SAGMS_OK;
}

int device_tables(Graph* g, DeviceTables** out) {
    int dev = 0;
    SAGMS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(SAGMS_EUNSUPPORTED, "device index %d too large", dev);
    std::lock_guard<std::mutex> lock(g->mu);
    DeviceTables* t = &g->dev[dev];
    if (!t->ready)
        return fail(SAGMS_EINVAL, "the graph has no tables on device %d: call sagms_graph_upload with it current", dev);
    *out = t;
    return SAGMS_OK;
}

}  // namespace sagms

using namespace sagms;

extern "C" {

const char* sagms_last_error(void) { return g_last_error.c_str(); }

int sagms_build_graph(int32_t m, int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t m_other,
                      const int32_t* row_ptr_o, const int32_t* col_idx_o, sagms_graph* out) {
    if (!out) return fail(SAGMS_EINVAL, "out is null");
    *out = nullptr;
    if (m < 1 || n < 1 || n > kMaxN) return fail(SAGMS_EINVAL, "need 1 <= m and 1 <= n <= %d (m=%d n=%d)", kMaxN, m, n);
    int rc = check_csr(m, n, row_ptr, col_idx, "H", true);
    if (rc) return rc;
    std::vector<int> rp(row_ptr, row_ptr + m + 1), ci(col_idx, col_idx + row_ptr[m]);
    std::vector<int> rpo, cio;
    if (m_other < 0) return fail(SAGMS_EINVAL, "m_other must be >= 0");
    if (m_other > 0) {
        rc = check_csr(m_other, n, row_ptr_o, col_idx_o, "H_other", false);
        if (rc) return rc;
        rpo.assign(row_ptr_o, row_ptr_o + m_other + 1);
        cio.assign(col_idx_o, col_idx_o + row_ptr_o[m_other]);
    }
    return build(m, n, rp, ci, m_other, rpo, cio, out);
}

static int check_gb(int32_t l, const int32_t* a, int32_t wa, const int32_t* b, int32_t wb) {
    if (l < 2 || 2 * l > kMaxN) return fail(SAGMS_EINVAL, "circulant size l=%d out of range", l);
    if (!a || !b || wa < 1 || wb < 1 || wa + wb < 2) return fail(SAGMS_EINVAL, "bad polynomial arguments");
    for (int t = 0; t < wa; ++t)
        if (a[t] < 0 || a[t] >= l) return fail(SAGMS_EINVAL, "exponent a[%d]=%d out of range", t, a[t]);
    for (int t = 0; t < wb; ++t)
        if (b[t] < 0 || b[t] >= l) return fail(SAGMS_EINVAL, "exponent b[%d]=%d out of range", t, b[t]);
    for (int s = 0; s < wa; ++s)
        for (int t = s + 1; t < wa; ++t)
            if (a[s] == a[t]) return fail(SAGMS_EINVAL, "repeated exponent in a");
    for (int s = 0; s < wb; ++s)
        for (int t = s + 1; t < wb; ++t)
            if (b[s] == b[t]) return fail(SAGMS_EINVAL, "repeated exponent in b");
    return SAGMS_OK;
}

int sagms_build_gb_joint(int32_t l, const int32_t* a, int32_t wa, const int32_t* b, int32_t wb, sagms_graph* out) {
    if (!out) return fail(SAGMS_EINVAL, "out is null");
    *out = nullptr;
    int rc = check_gb(l, a, wa, b, wb);
    if (rc) return rc;
    Graph* g = new (std::nothrow) Graph();
    if (!g) return fail(SAGMS_ENOMEM, "graph allocation failed");
    g->joint = true;
    g->is_gb = true;
    g->gb_l = l;
    g->gb_a.assign(a, a + wa);
    g->gb_b.assign(b, b + wb);
    g->m = 2 * l;
    g->n = 2 * l;
    // X-type check c: row c of H_X = [A | B], columns (c + a_t) mod l and
    // l + (c + b_t) mod l; Z-type check l + c: row c of H_Z = [B^T | A^T],
    // columns (c - b_t) mod l and l + (c - a_t) mod l (term order)
    g->row_ptr.assign(2 * l + 1, 0);
    for (int c = 0; c < l; ++c) {
        g->row_ptr[c] = (int)g->cols.size();
        for (int t = 0; t < wa; ++t) g->cols.push_back((c + a[t]) % l);
        for (int t = 0; t < wb; ++t) g->cols.push_back(l + (c + b[t]) % l);
    }
    for (int c = 0; c < l; ++c) {
        g->row_ptr[l + c] = (int)g->cols.size();
        for (int t = 0; t < wb; ++t) g->cols.push_back(((c - b[t]) % l + l) % l);
        for (int t = 0; t < wa; ++t) g->cols.push_back(l + ((c - a[t]) % l + l) % l);
    }
    g->row_ptr[2 * l] = (int)g->cols.size();
    rc = finish_joint(g);
    if (rc != SAGMS_OK) {
        delete g;
        return rc;
    }
    return publish(g, out);
}

int sagms_build_gb(int32_t l, const int32_t* a, int32_t wa, const int32_t* b, int32_t wb, sagms_graph* out) {
    if (!out) return fail(SAGMS_EINVAL, "out is null");
    *out = nullptr;
    int rc = check_gb(l, a, wa, b, wb);
    if (rc) return rc;
    // H_Z = [B^T | A^T]: row c has ones at (c - b_t) mod l and l + (c - a_t) mod l.
    // Edge positions follow the polynomial terms, so that lanes reading the
    // same position touch consecutive posteriors (the order does not change
    // any result: the check update is symmetric in its inputs).
    std::vector<int> rp(l + 1), ci;
    for (int c = 0; c < l; ++c) {
        rp[c] = (int)ci.size();
        for (int t = 0; t < wb; ++t) ci.push_back(((c - b[t]) % l + l) % l);
        for (int t = 0; t < wa; ++t) ci.push_back(l + ((c - a[t]) % l + l) % l);
    }
    rp[l] = (int)ci.size();
    // H_X = [A | B]: row c has ones at (c + a_t) mod l and l + (c + b_t) mod l.
    std::vector<int> rpo(l + 1), cio;
    for (int c = 0; c < l; ++c) {
        rpo[c] = (int)cio.size();
        for (int t = 0; t < wa; ++t) cio.push_back((c + a[t]) % l);
        for (int t = 0; t < wb; ++t) cio.push_back(l + (c + b[t]) % l);
    }
    rpo[l] = (int)cio.size();
    std::vector<int> va(a, a + wa), vb(b, b + wb);
    return build(l, 2 * l, rp, ci, l, rpo, cio, out, &va, &vb);
}

int sagms_graph_info(sagms_graph gh, sagms_graph_info_t* info) {
    Graph* g = reinterpret_cast<Graph*>(gh);
    if (!g || !info) return fail(SAGMS_EINVAL, "null argument");
    info->m = g->m;
    info->n = g->n;
    info->n_edges = g->E;
    info->k = g->have_other ? g->k : -1;
    info->dc_max = g->dc_max;
    info->dv_max = g->dv_max;
    info->words_n = g->wn;
    info->words_m = g->wm;
    info->joint = g->joint ? 1 : 0;
    info->words_e = g->we;
    const bool layered = g->layered.status == SAGMS_OK;
    info->layered_group = layered ? g->layered.group : 0;
    info->layered_passes = layered ? g->layered.passes : 0;
    return SAGMS_OK;
}

int sagms_graph_rows(sagms_graph gh, uint64_t* rows) {
    Graph* g = reinterpret_cast<Graph*>(gh);
    if (!g || !rows) return fail(SAGMS_EINVAL, "null argument");
    std::memcpy(rows, g->rows_bits.data(), g->rows_bits.size() * sizeof(uint64_t));
    return SAGMS_OK;
}

int sagms_graph_logicals(sagms_graph gh, uint64_t* rows) {
    Graph* g = reinterpret_cast<Graph*>(gh);
    if (!g || !rows) return fail(SAGMS_EINVAL, "null argument");
    if (!g->have_other) return fail(SAGMS_EINVAL, "graph has no other matrix");
    std::memcpy(rows, g->logicals.data(), g->logicals.size() * sizeof(uint64_t));
    return SAGMS_OK;
}

int sagms_destroy_graph(sagms_graph gh) {
    Graph* g = reinterpret_cast<Graph*>(gh);
    if (!g) return fail(SAGMS_EINVAL, "null graph");
    int cur = -1;
    bool have_dev = hipGetDevice(&cur) == hipSuccess;
    for (int d = 0; d < kMaxDevices; ++d) {
        DeviceTables& t = g->dev[d];
        if (!t.ready) continue;
        if (have_dev) (void)hipSetDevice(d);
        free_tables(&t);
    }
    if (have_dev) (void)hipSetDevice(cur);
    delete g;
    return SAGMS_OK;
}

int sagms_graph_upload(sagms_graph gh) {
    Graph* g = reinterpret_cast<Graph*>(gh);
    if (!g) return fail(SAGMS_EINVAL, "null graph");
    DeviceTables* t = nullptr;
    return upload_tables(g, &t);
}

double sagms_alpha_star(double l0, int32_t dc) {
    if (!(l0 > 0.0) || dc < 2) return std::nan("");
    // y = tanh(L0/2)^(dc-1) from log tanh(L0/2) = log1p(-2 / (e^L0 + 1));
    // 2 atanh(y) = log1p(y) - log(1 - y), with 1 - y = -expm1((dc-1) log tanh)
    // kept exact near y = 1 and log1p(-y) used for small y
    const double lt = std::log1p(-2.0 / (std::exp(l0) + 1.0));
    const double y = std::exp((dc - 1) * lt);
    const double one_minus_y = -std::expm1((dc - 1) * lt);
    if (!(one_minus_y > 0.0)) return 1.0;  // y rounds to 1 only as L0 -> inf, where alpha* -> 1
    const double two_atanh = std::log1p(y) - (y < 0.5 ? std::log1p(-y) : std::log(one_minus_y));
    return two_atanh / l0;
}

int sagms_derive_gains(double l0, int32_t dc, double ratio, double eta, sagms_decoder_cfg* cfg) {
    if (!cfg) return fail(SAGMS_EINVAL, "cfg is null");
    if (!(l0 > 0.0) || dc < 2) return fail(SAGMS_EINVAL, "need L0 > 0 and d_c >= 2");
    if (!(ratio > 0.0 && ratio <= 1.0)) return fail(SAGMS_EINVAL, "ratio must lie in (0, 1]");
    const double amax = sagms_alpha_star(l0, dc);
    double e = eta;
    if (!(eta > 0.0)) {
        e = 1.0 / amax;
        while (amax * e > 1.0) e = std::nextafter(e, 0.0);  // the largest eta with alpha_max * eta <= 1
    }
    if (!(amax * e <= 1.0)) return fail(SAGMS_EINVAL, "alpha_max * eta = %g exceeds 1", amax * e);
    if (!(e >= 1.0)) return fail(SAGMS_EINVAL, "eta must be >= 1");
    cfg->kind = SAGMS_SAGMS;
    cfg->alpha_max = amax;
    cfg->alpha_min = ratio * amax;
    cfg->eta = e;
    return SAGMS_OK;
}

float sagms_depolarizing_llr(double p) {
    if (!(p > 0.0 && p < 0.75)) return NAN;
    return (float)std::log((1.0 - p) / (p / 3.0));
}

float sagms_prior_llr(double p) {
    if (!(p > 0.0 && p < 0.75)) return NAN;
    double q = 2.0 * p / 3.0;
    return (float)std::log((1.0 - q) / q);
}

}  // extern "C"
