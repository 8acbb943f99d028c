// Patch plan of one mesh (host, set-up time only).
//
// The element restriction R and its transpose (the G/G^T of the paper's
// operator decomposition, Sec. 3.1) are applied per patch: a set of
// neighbouring elements handled by one workgroup. Elements are ordered along a
// Morton curve of their centroids so that consecutive elements are neighbours,
// then cut greedily into patches of at most B elements and at most UMAX
// distinct nodes. Within a patch every distinct node gets an LDS slot; element
// results are accumulated there, and R^T becomes
//   - a plain store for nodes touched by this patch only ("private" nodes),
//   - a write of the patch's partial sum for nodes shared with other patches,
//     followed by a gather that adds the partials of each shared node in a
//     fixed order.
#include "patch.hpp"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>

namespace fepa {

static uint64_t spread3(uint64_t v)
{
    v &= 0x1fffff;
    v = (v | v << 32) & 0x1f00000000ffffULL;
    v = (v | v << 16) & 0x1f0000ff0000ffULL;
    v = (v | v << 8) & 0x100f00f00f00f00fULL;
    v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
    v = (v | v << 2) & 0x1249249249249249ULL;
    return v;
}

PatchPlan build_patch_plan(int E, int p, int N, const int32_t *map, const double *x0, int B,
                           int umax)
{
    const int D = p + 1, D3 = D * D * D;
    PatchPlan pl;
    // element centroids from the 8 vertex nodes
    std::vector<double> cen(3 * (size_t)E);
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int el = 0; el < E; ++el) {
        double c[3] = {0, 0, 0};
        for (int cz = 0; cz < 2; ++cz)
            for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx) {
                    const int i = cx * p + D * (cy * p + D * cz * p);
                    const int32_t g = map[(size_t)el * D3 + i];
                    for (int k = 0; k < 3; ++k) c[k] += 0.125 * x0[(size_t)k * N + g];
                }
        for (int k = 0; k < 3; ++k) {
            cen[3 * (size_t)el + k] = c[k];
            lo[k] = std::min(lo[k], c[k]);
            hi[k] = std::max(hi[k], c[k]);
        }
    }
    // quantise on the mean element size, then Morton-sort
    double vol = 1.0;
    for (int k = 0; k < 3; ++k) vol *= std::max(hi[k] - lo[k], 1e-300);
    double h = std::cbrt(vol / E);
    if (!(h > 0.0)) h = 1.0;
    std::vector<uint64_t> code(E);
    for (int el = 0; el < E; ++el) {
        uint64_t q[3];
        for (int k = 0; k < 3; ++k) {
            double t = std::floor((cen[3 * (size_t)el + k] - lo[k]) / h + 0.5);
            t = std::min(std::max(t, 0.0), 2097151.0);
            q[k] = (uint64_t)t;
        }
        code[el] = spread3(q[0]) | spread3(q[1]) << 1 | spread3(q[2]) << 2;
    }
    pl.perm.resize(E);
    std::iota(pl.perm.begin(), pl.perm.end(), 0);
    std::stable_sort(pl.perm.begin(), pl.perm.end(),
                     [&](int a, int b) { return code[a] < code[b]; });

    // greedy patches along the curve
    std::vector<int> stamp(N, -1), cnt(N, 0);
    std::vector<int32_t> tmp;
    int cur = -1, U = 0, n_in = 0;
    for (int k = 0; k < E; ++k) {
        const int32_t *row = map + (size_t)pl.perm[k] * D3;
        int fresh = D3;
        if (cur >= 0) {
            tmp.clear();
            for (int i = 0; i < D3; ++i)
                if (stamp[row[i]] != cur) tmp.push_back(row[i]);
            std::sort(tmp.begin(), tmp.end());
            fresh = (int)(std::unique(tmp.begin(), tmp.end()) - tmp.begin());
        }
        if (cur < 0 || n_in == B || U + fresh > umax) {
            pl.patch.push_back(PatchRec{k, 0, 0, 0, 0, 0});
            cur = (int)pl.patch.size() - 1;
            U = 0;
            n_in = 0;
        }
        for (int i = 0; i < D3; ++i)
            if (stamp[row[i]] != cur) {
                stamp[row[i]] = cur;
                ++cnt[row[i]];
                ++U;
            }
        ++n_in;
        pl.patch[cur].count = n_in;
        pl.patch[cur].U = U;
    }
    // per patch: distinct nodes, private first, then shared; slots per element node
    pl.slot.resize((size_t)E * D3);
    pl.map_int.resize((size_t)E * D3);
    std::vector<int> where(N, -1), slot_of(N, -1);
    std::vector<int32_t> priv, shar;
    int n_entries = 0;
    std::vector<std::pair<int32_t, int32_t>> entries;  // (node, entry index)
    for (size_t k = 0; k < pl.patch.size(); ++k) {
        PatchRec &pr = pl.patch[k];
        priv.clear();
        shar.clear();
        for (int e = pr.elem_begin; e < pr.elem_begin + pr.count; ++e) {
            const int32_t *row = map + (size_t)pl.perm[e] * D3;
            for (int i = 0; i < D3; ++i) {
                const int32_t g = row[i];
                if (where[g] == (int)k) continue;
                where[g] = (int)k;
                (cnt[g] == 1 ? priv : shar).push_back(g);
            }
        }
        std::sort(priv.begin(), priv.end());
        std::sort(shar.begin(), shar.end());
        pr.pn_off = (int)pl.pn.size();
        pr.P = (int)priv.size();
        pr.U = (int)(priv.size() + shar.size());
        pr.sh_off = n_entries;
        pl.pn.insert(pl.pn.end(), priv.begin(), priv.end());
        pl.pn.insert(pl.pn.end(), shar.begin(), shar.end());
        for (size_t j = 0; j < shar.size(); ++j) entries.emplace_back(shar[j], n_entries + (int)j);
        n_entries += (int)shar.size();
        for (int u = 0; u < pr.U; ++u) slot_of[pl.pn[pr.pn_off + u]] = u;
        for (int e = pr.elem_begin; e < pr.elem_begin + pr.count; ++e) {
            const int32_t *row = map + (size_t)pl.perm[e] * D3;
            for (int i = 0; i < D3; ++i) {
                pl.slot[(size_t)e * D3 + i] = (uint16_t)slot_of[row[i]];
                pl.map_int[(size_t)e * D3 + i] = row[i];
            }
        }
        for (int u = 0; u < pr.U; ++u) slot_of[pl.pn[pr.pn_off + u]] = -1;
        pl.umax_used = std::max(pl.umax_used, pr.U);
    }
    // shared-node gather lists, entries of a node in ascending patch order
    std::stable_sort(entries.begin(), entries.end(),
                     [](const std::pair<int32_t, int32_t> &a, const std::pair<int32_t, int32_t> &b) {
                         return a.first < b.first;
                     });
    pl.n_entries = n_entries;
    pl.sh_ptr.push_back(0);
    for (size_t j = 0; j < entries.size(); ++j) {
        if (j == 0 || entries[j].first != entries[j - 1].first) {
            if (j) pl.sh_ptr.push_back((int32_t)j);
            pl.sh_node.push_back(entries[j].first);
        }
        pl.sh_idx.push_back(entries[j].second);
    }
    if (!entries.empty()) pl.sh_ptr.push_back((int32_t)entries.size());
    for (int g = 0; g < N; ++g)
        if (cnt[g] == 0) pl.orphans.push_back(g);
    return pl;
}

void append_plan(PatchPlan &dst, const PatchPlan &src, int32_t perm_base)
{
    const int e0 = (int)dst.perm.size(), pn0 = (int)dst.pn.size(), en0 = dst.n_entries;
    const int idx0 = (int)dst.sh_idx.size();
    for (int32_t g : src.perm) dst.perm.push_back(g + perm_base);
    dst.map_int.insert(dst.map_int.end(), src.map_int.begin(), src.map_int.end());
    dst.slot.insert(dst.slot.end(), src.slot.begin(), src.slot.end());
    dst.pn.insert(dst.pn.end(), src.pn.begin(), src.pn.end());
    for (PatchRec r : src.patch) {
        r.elem_begin += e0;
        r.pn_off += pn0;
        r.sh_off += en0;
        dst.patch.push_back(r);
    }
    if (dst.sh_ptr.empty()) dst.sh_ptr.push_back(0);
    dst.sh_node.insert(dst.sh_node.end(), src.sh_node.begin(), src.sh_node.end());
    for (size_t k = 1; k < src.sh_ptr.size(); ++k) dst.sh_ptr.push_back(src.sh_ptr[k] + idx0);
    for (int32_t j : src.sh_idx) dst.sh_idx.push_back(j + en0);
    dst.orphans.insert(dst.orphans.end(), src.orphans.begin(), src.orphans.end());
    dst.n_entries += src.n_entries;
    dst.umax_used = std::max(dst.umax_used, src.umax_used);
}

}  // namespace fepa
