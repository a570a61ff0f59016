// pic_tree.hip -- host construction of the linearised spacetree forest.
//
// A k = 3 spacetree (paper Sec. 4) is stored as flat arrays:
//  * a level-major descent table: each refined, non-uniform node points at its
//    3^d children (lexicographic child slots, so a child is found by index
//    arithmetic); a node whose leaves all sit on one level ("uniform subtree",
//    a regular tree's root being the extreme case) ends the descent and its
//    leaves are ranked arithmetically by the Peano rank of their coordinates;
//  * leaves ranked by their Peano key (the storage order of Sec. 4.2), with
//    their level, corner vertices and corner dual cells;
//  * vertices = distinct leaf-corner positions (hanging ones included),
//    numbered lexicographically per instance;
//  * dual-grid bins (PIDT, Sec. 4.1 and 5.2) = (level, vertex of a leaf of that
//    level), keyed on the half-cell-shifted lattice on which dual cells nest
//    for odd k.
#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "pic_host.h"

namespace pic {

static uint64_t peano64(int dim, const uint32_t *a, int nd) {
    // 64-bit variant of peano_low for full-depth keys (dim * nd <= 36 digits)
    uint32_t q[3] = {a[0], a[1], dim > 2 ? a[2] : 0u};
    uint64_t key = 0, mult = 1;
    for (int t = 0; t < nd; ++t) {
        uint32_t qn[3], dig[3];
        for (int k = 0; k < dim; ++k) {
            qn[k] = q[k] / 3u;
            dig[k] = q[k] - 3u * qn[k];
        }
        for (int k = dim - 1; k >= 0; --k) {
            uint32_t par = 0;
            for (int j = 0; j < dim; ++j) {
                if (j < k) par ^= q[j] & 1u;
                else if (j > k) par ^= qn[j] & 1u;
            }
            uint64_t e = par ? 2u - dig[k] : dig[k];
            key += e * mult;
            mult *= 3u;
        }
        for (int k = 0; k < dim; ++k) q[k] = qn[k];
    }
    return key;
}

uint64_t host_peano(int dim, const uint32_t *a, int nd) { return peano64(dim, a, nd); }

namespace {

struct FullNode {
    int32_t level;
    uint32_t a[3];
    int32_t first_child;  // -1 for a leaf
};

}  // namespace

pic_status build_instance(int dim, int L, const uint8_t *masks, HostInst &out) {
    const int nch = dim == 2 ? 9 : 27;
    const int nc = 1 << dim;
    const int64_t S = (int64_t)pow3_u64(L);
    out = HostInst();
    out.L = L;
    out.S = S;

    // 1. full level-major node list from the masks
    std::vector<FullNode> nodes;
    std::vector<int64_t> level_begin(L + 2, 0);
    nodes.push_back(FullNode{0, {0, 0, 0}, -1});
    level_begin[1] = 1;
    int64_t mask_off = 0;
    for (int l = 0; l < L; ++l) {
        const int64_t n_l = (int64_t)pow3_u64(l);
        const int64_t cells = dim == 2 ? n_l * n_l : n_l * n_l * n_l;
        for (int64_t i = level_begin[l]; i < level_begin[l + 1]; ++i) {
            const uint32_t a[3] = {nodes[i].a[0], nodes[i].a[1], nodes[i].a[2]};  // copy: push_back reallocates
            int64_t lex = a[0] + n_l * (a[1] + (dim > 2 ? n_l * (int64_t)a[2] : 0));
            if (!masks[mask_off + lex]) continue;
            nodes[i].first_child = (int32_t)nodes.size();
            for (int s = 0; s < nch; ++s) {
                FullNode c{l + 1, {3 * a[0] + s % 3, 3 * a[1] + (s / 3) % 3,
                                   dim > 2 ? 3 * a[2] + s / 9 : 0u}, -1};
                nodes.push_back(c);
            }
            if ((int64_t)nodes.size() > (int64_t)INT32_MAX / 2) return PIC_E_TREE;
        }
        level_begin[l + 2] = (int64_t)nodes.size();
        mask_off += cells;
    }
    const int64_t n_full = (int64_t)nodes.size();

    // 2. leaves in Peano-key order
    std::vector<int64_t> leaf_nodes;
    for (int64_t i = 0; i < n_full; ++i)
        if (nodes[i].first_child < 0) leaf_nodes.push_back(i);
    const int64_t nl = (int64_t)leaf_nodes.size();
    std::vector<uint64_t> key(nl);
    for (int64_t r = 0; r < nl; ++r) {
        const FullNode &n = nodes[leaf_nodes[r]];
        uint64_t span = pow3_u64(dim * (L - n.level));
        key[r] = peano64(dim, n.a, n.level) * span * 64u + (uint64_t)n.level;
    }
    std::vector<int64_t> order(nl);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int64_t x, int64_t y) { return key[x] < key[y]; });
    std::vector<int32_t> node_rank(n_full, -1);
    out.leaf_key.resize(nl);
    out.leaf_level.resize(nl);
    out.leaf_coord.resize(nl * dim);
    for (int64_t r = 0; r < nl; ++r) {
        int64_t id = leaf_nodes[order[r]];
        node_rank[id] = (int32_t)r;
        out.leaf_key[r] = key[order[r]];
        out.leaf_level[r] = (uint8_t)nodes[id].level;
        for (int k = 0; k < dim; ++k) out.leaf_coord[r * dim + k] = nodes[id].a[k];
    }

    // 3. per node: leaf-level range and first leaf rank of its subtree (bottom-up)
    std::vector<int32_t> lmin(n_full), lmax(n_full), rmin(n_full);
    for (int64_t i = n_full - 1; i >= 0; --i) {
        if (nodes[i].first_child < 0) {
            lmin[i] = lmax[i] = nodes[i].level;
            rmin[i] = node_rank[i];
        } else {
            int64_t c0 = nodes[i].first_child;
            lmin[i] = lmin[c0];
            lmax[i] = lmax[c0];
            rmin[i] = rmin[c0];
            for (int s = 1; s < nch; ++s) {
                lmin[i] = std::min(lmin[i], lmin[c0 + s]);
                lmax[i] = std::max(lmax[i], lmax[c0 + s]);
                rmin[i] = std::min(rmin[i], rmin[c0 + s]);
            }
        }
    }
    out.regular = (lmin[0] == L && lmax[0] == L) ? 1 : 0;

    // 4. compacted descent table: breadth-first, stopping at uniform nodes
    {
        std::vector<int64_t> cur{0}, next;
        while (!cur.empty()) {
            next.clear();
            int64_t base = (int64_t)out.node_child.size() + (int64_t)cur.size();
            for (int64_t id : cur) {
                if (lmin[id] == lmax[id]) {
                    int32_t u = (int32_t)out.uni_base.size();
                    out.uni_base.push_back((uint32_t)rmin[id]);
                    out.uni_meta.push_back((uint32_t)nodes[id].level |
                                           ((uint32_t)(lmax[id] - nodes[id].level) << 8));
                    out.node_child.push_back(-(u + 1));
                } else {
                    out.node_child.push_back((int32_t)(base + (int64_t)next.size()));
                    for (int s = 0; s < nch; ++s) next.push_back(nodes[id].first_child + s);
                }
            }
            cur.swap(next);
        }
    }

    // 5. vertices: distinct corner positions, lexicographic (axis 0 fastest)
    std::vector<int64_t> lin(nl * nc);
    for (int64_t r = 0; r < nl; ++r) {
        int lv = out.leaf_level[r];
        int64_t s = (int64_t)pow3_u64(L - lv);
        for (int c = 0; c < nc; ++c) {
            int64_t v = 0, m = 1;
            for (int k = 0; k < dim; ++k) {
                int64_t p = (((int64_t)out.leaf_coord[r * dim + k] + ((c >> k) & 1)) * s) % S;
                v += p * m;
                m *= S;
            }
            lin[r * nc + c] = v;
        }
    }
    out.vtx_lin = lin;
    std::sort(out.vtx_lin.begin(), out.vtx_lin.end());
    out.vtx_lin.erase(std::unique(out.vtx_lin.begin(), out.vtx_lin.end()), out.vtx_lin.end());
    out.leaf_vtx.resize(nl * nc);
    for (int64_t i = 0; i < nl * nc; ++i)
        out.leaf_vtx[i] = (int32_t)(std::lower_bound(out.vtx_lin.begin(), out.vtx_lin.end(), lin[i]) -
                                    out.vtx_lin.begin());

    // 6. dual-grid bins
    std::vector<uint64_t> pk(nl * nc);
    for (int64_t r = 0; r < nl; ++r) {
        int lv = out.leaf_level[r];
        int64_t s = (int64_t)pow3_u64(L - lv), nlv = (int64_t)pow3_u64(lv);
        for (int c = 0; c < nc; ++c) {
            uint32_t J[3] = {0, 0, 0};
            for (int k = 0; k < dim; ++k) {
                int64_t b = ((int64_t)out.leaf_coord[r * dim + k] + ((c >> k) & 1)) % nlv;
                J[k] = (uint32_t)((b * s + (S - 1) / 2) % S);
            }
            pk[r * nc + c] = peano64(dim, J, L) * 64u + (uint64_t)lv;
        }
    }
    out.pidt_key = pk;
    std::sort(out.pidt_key.begin(), out.pidt_key.end());
    out.pidt_key.erase(std::unique(out.pidt_key.begin(), out.pidt_key.end()), out.pidt_key.end());
    const int64_t np = (int64_t)out.pidt_key.size();
    out.leaf_pidt.resize(nl * nc);
    out.pidt_level.resize(np);
    out.pidt_b.resize(np * dim);
    out.pidt_vtx.resize(np);
    for (int64_t r = 0; r < nl; ++r) {
        int lv = out.leaf_level[r];
        int64_t nlv = (int64_t)pow3_u64(lv);
        for (int c = 0; c < nc; ++c) {
            int32_t bin = (int32_t)(std::lower_bound(out.pidt_key.begin(), out.pidt_key.end(), pk[r * nc + c]) -
                                    out.pidt_key.begin());
            out.leaf_pidt[r * nc + c] = bin;
            out.pidt_level[bin] = (uint8_t)lv;
            for (int k = 0; k < dim; ++k)
                out.pidt_b[bin * dim + k] = (uint32_t)(((int64_t)out.leaf_coord[r * dim + k] + ((c >> k) & 1)) % nlv);
            out.pidt_vtx[bin] = out.leaf_vtx[r * nc + c];
        }
    }
    if (nl > INT32_MAX / 32 || (int64_t)out.vtx_lin.size() > INT32_MAX / 32 || np > INT32_MAX / 32)
        return PIC_E_TREE;
    return PIC_OK;
}

// CSR incidence tables for adaptive instances (regular ones are handled by
// arithmetic in the kernels and get empty rows).
void build_incidence(int dim, const HostInst &h, int32_t leaf_off, int32_t pidt_off,
                     std::vector<std::vector<int32_t>> &vinc_rows,
                     std::vector<std::vector<int32_t>> &vpinc_rows) {
    const int nc = 1 << dim;
    const int nsten = dim == 2 ? 9 : 27;
    const int64_t nl = (int64_t)h.leaf_level.size();
    const int64_t nv = (int64_t)h.vtx_lin.size();
    vinc_rows.assign(nv, {});
    vpinc_rows.assign(nv, {});
    for (int64_t r = 0; r < nl; ++r)
        for (int c = 0; c < nc; ++c)
            vinc_rows[h.leaf_vtx[r * nc + c]].push_back((int32_t)((leaf_off + r) * nc + c));
    // PIDT stencil: a particle owned by corner o of leaf r deposits on every
    // corner c of r, i.e. on stencil slot sum_k (c_k - o_k + 1) 3^k of bin(o)
    for (int64_t r = 0; r < nl; ++r)
        for (int o = 0; o < nc; ++o) {
            int32_t bin = h.leaf_pidt[r * nc + o];
            for (int c = 0; c < nc; ++c) {
                int slot = 0, m = 1;
                for (int k = 0; k < dim; ++k) {
                    slot += (((c >> k) & 1) - ((o >> k) & 1) + 1) * m;
                    m *= 3;
                }
                vpinc_rows[h.leaf_vtx[r * nc + c]].push_back((int32_t)((int64_t)(pidt_off + bin) * nsten + slot));
            }
        }
    for (auto &row : vinc_rows) std::sort(row.begin(), row.end());
    for (auto &row : vpinc_rows) {
        std::sort(row.begin(), row.end());
        row.erase(std::unique(row.begin(), row.end()), row.end());
    }
}

}  // namespace pic
