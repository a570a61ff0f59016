// pic_capi.hip -- the extern "C" boundary (include/pic.h): argument checks,
// forest assembly, the device image of the tree, and launch sequencing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <new>
#include <string>

#include "pic_host.h"

using namespace pic;

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

bool valid_scheme(int32_t s) { return s == PIC_PIT || s == PIC_PIDT; }

template <typename T>
void put(std::vector<uint8_t> &img, int64_t off, const T *src, int64_t count) {
    if (count > 0) std::memcpy(img.data() + off, src, (size_t)count * sizeof(T));
}

// Lay out the device image and fill the host copy.
pic_status assemble(pic_tree *t) {
    const int dim = t->dim;
    const int nc = 1 << dim;
    const int nsten = dim == 2 ? 9 : 27;
    const int ni = t->n_inst;
    t->leaf_off.assign(ni + 1, 0);
    t->vtx_off.assign(ni + 1, 0);
    t->pidt_off.assign(ni + 1, 0);
    t->node_off.assign(ni + 1, 0);
    std::vector<int64_t> uni_off(ni + 1, 0);
    for (int i = 0; i < ni; ++i) {
        const HostInst &h = t->inst[i];
        t->leaf_off[i + 1] = t->leaf_off[i] + (int64_t)h.leaf_level.size();
        t->vtx_off[i + 1] = t->vtx_off[i] + (int64_t)h.vtx_lin.size();
        t->pidt_off[i + 1] = t->pidt_off[i] + (int64_t)h.pidt_key.size();
        t->node_off[i + 1] = t->node_off[i] + (int64_t)h.node_child.size();
        uni_off[i + 1] = uni_off[i] + (int64_t)h.uni_base.size();
    }
    const int64_t NL = t->leaf_off[ni], NV = t->vtx_off[ni], NP = t->pidt_off[ni], NN = t->node_off[ni],
                  NU = uni_off[ni];
    if (NL >= INT32_MAX / 32 || NV >= INT32_MAX / 32 || NP >= INT32_MAX / 32 || NN >= INT32_MAX)
        return PIC_E_TREE;
    t->n_nodes = NN;

    // incidence lists for adaptive instances
    std::vector<int32_t> vptr(NV + 1, 0), vpptr(NV + 1, 0), vinc, vpinc;
    if (!t->all_regular) {
        for (int i = 0; i < ni; ++i) {
            const HostInst &h = t->inst[i];
            if (h.regular) continue;
            std::vector<std::vector<int32_t>> rows, prows;
            build_incidence(dim, h, (int32_t)t->leaf_off[i], (int32_t)t->pidt_off[i], rows, prows);
            for (size_t v = 0; v < rows.size(); ++v) {
                vptr[t->vtx_off[i] + v + 1] = (int32_t)rows[v].size();
                vpptr[t->vtx_off[i] + v + 1] = (int32_t)prows[v].size();
            }
            // rows are appended in vertex order below
            for (auto &r : rows) vinc.insert(vinc.end(), r.begin(), r.end());
            for (auto &r : prows) vpinc.insert(vpinc.end(), r.begin(), r.end());
        }
        // vinc/vpinc were appended instance by instance in vertex order; turn counts into offsets
        for (int64_t v = 0; v < NV; ++v) {
            vptr[v + 1] += vptr[v];
            vpptr[v + 1] += vpptr[v];
        }
    }
    t->n_vinc = (int64_t)vinc.size();
    t->n_vpinc = (int64_t)vpinc.size();

    // Peano rank tables for the levels of regular instances (shared by
    // instances of equal level), when a level's table is small enough
    constexpr int64_t kMaxTab = int64_t(1) << 21;
    std::vector<int64_t> tab_off(PIC_MAX_LEVEL + 1, -1);
    std::vector<uint32_t> ptab;
    for (int i = 0; i < ni; ++i) {
        const HostInst &h = t->inst[i];
        if (!g_tune.regular_tables || !h.regular || tab_off[h.L] >= 0) continue;
        int64_t cells = 1;
        for (int k = 0; k < dim; ++k) cells *= (int64_t)h.S;
        if (cells > kMaxTab) continue;
        tab_off[h.L] = (int64_t)ptab.size();
        ptab.resize(ptab.size() + (size_t)cells);
        uint32_t *dst = ptab.data() + tab_off[h.L];
        const uint32_t S = (uint32_t)h.S;
        for (int64_t c = 0; c < cells; ++c) {
            uint32_t a[3] = {(uint32_t)(c % S), (uint32_t)((c / S) % S), (uint32_t)(c / ((int64_t)S * S))};
            dst[c] = dim == 2 ? peano_low<2>(a, h.L) : peano_low<3>(a, h.L);
        }
    }
    std::vector<uint32_t> ctab(ptab.size());
    for (int l = 0; l <= PIC_MAX_LEVEL; ++l) {
        if (tab_off[l] < 0) continue;
        int64_t cells = 1;
        for (int k = 0; k < dim; ++k) cells *= (int64_t)pow3_u64(l);
        for (int64_t c = 0; c < cells; ++c) ctab[tab_off[l] + ptab[tab_off[l] + c]] = (uint32_t)c;
    }

    size_t o = 0;
    t->o_status = o; o = align256(o + 256);
    t->o_inst = o; o = align256(o + (size_t)ni * sizeof(DevInst));
    t->o_node = o; o = align256(o + (size_t)NN * 4);
    t->o_ubase = o; o = align256(o + (size_t)NU * 4);
    t->o_umeta = o; o = align256(o + (size_t)NU * 4);
    t->o_llev = o; o = align256(o + (size_t)NL);
    t->o_lvtx = o; o = align256(o + (size_t)NL * nc * 4);
    t->o_lpidt = o; o = align256(o + (size_t)NL * nc * 4);
    t->o_plev = o; o = align256(o + (size_t)NP);
    t->o_linst = o; o = align256(o + (size_t)NL * 4);
    t->o_pinst = o; o = align256(o + (size_t)NP * 4);
    t->o_vinst = o; o = align256(o + (size_t)NV * 4);
    t->o_vptr = o; o = align256(o + (size_t)(NV + 1) * 4);
    t->o_vinc = o; o = align256(o + (size_t)vinc.size() * 4);
    t->o_vpptr = o; o = align256(o + (size_t)(NV + 1) * 4);
    t->o_vpinc = o; o = align256(o + (size_t)vpinc.size() * 4);
    t->o_ptab = o; o = align256(o + ptab.size() * 4);
    t->o_ctab = o; o = align256(o + ctab.size() * 4);
    t->o_lcoord = o; o = align256(o + (size_t)NL * dim * 4);
    t->o_pb = o; o = align256(o + (size_t)NP * dim * 4);
    t->device_bytes = (int64_t)o;
    t->image.assign(o, 0);

    std::vector<DevInst> di(ni);
    for (int i = 0; i < ni; ++i) {
        const HostInst &h = t->inst[i];
        DevInst &d = di[i];
        std::memset(&d, 0, sizeof(d));
        d.L = h.L;
        d.regular = h.regular;
        d.S = (int32_t)h.S;
        d.node_root = (int32_t)t->node_off[i];
        d.leaf_off = (int32_t)t->leaf_off[i];
        d.n_leaves = (int32_t)h.leaf_level.size();
        d.vtx_off = (int32_t)t->vtx_off[i];
        d.n_vtx = (int32_t)h.vtx_lin.size();
        d.pidt_off = (int32_t)t->pidt_off[i];
        d.n_pidt = (int32_t)h.pidt_key.size();
        d.lds_nodes = (int32_t)std::min<int64_t>((int64_t)h.node_child.size(), PIC_LDS_NODES);
        d.ptab = h.regular ? (int32_t)tab_off[h.L] : -1;
        d.Sd = (double)h.S;
        for (int l = 0; l <= h.L; ++l) d.rinv[l] = 1.0 / (double)pow3_u64(h.L - l);
        // node table with forest-wide indices
        std::vector<int32_t> nodes(h.node_child.size());
        for (size_t j = 0; j < nodes.size(); ++j) {
            int32_t c = h.node_child[j];
            nodes[j] = c >= 0 ? c + (int32_t)t->node_off[i] : -((-c - 1) + (int32_t)uni_off[i] + 1);
        }
        put(t->image, t->o_node + t->node_off[i] * 4, nodes.data(), (int64_t)nodes.size());
        std::vector<uint32_t> ub(h.uni_base.size());
        for (size_t j = 0; j < ub.size(); ++j) ub[j] = h.uni_base[j] + (uint32_t)t->leaf_off[i];
        put(t->image, t->o_ubase + uni_off[i] * 4, ub.data(), (int64_t)ub.size());
        put(t->image, t->o_umeta + uni_off[i] * 4, h.uni_meta.data(), (int64_t)h.uni_meta.size());
        put(t->image, t->o_llev + t->leaf_off[i], h.leaf_level.data(), (int64_t)h.leaf_level.size());
        std::vector<int32_t> lv(h.leaf_vtx.size()), lp(h.leaf_pidt.size());
        for (size_t j = 0; j < lv.size(); ++j) lv[j] = h.leaf_vtx[j] + (int32_t)t->vtx_off[i];
        for (size_t j = 0; j < lp.size(); ++j) lp[j] = h.leaf_pidt[j] + (int32_t)t->pidt_off[i];
        put(t->image, t->o_lvtx + t->leaf_off[i] * nc * 4, lv.data(), (int64_t)lv.size());
        put(t->image, t->o_lpidt + t->leaf_off[i] * nc * 4, lp.data(), (int64_t)lp.size());
        put(t->image, t->o_plev + t->pidt_off[i], h.pidt_level.data(), (int64_t)h.pidt_level.size());
        put(t->image, t->o_lcoord + t->leaf_off[i] * dim * 4, h.leaf_coord.data(), (int64_t)h.leaf_coord.size());
        put(t->image, t->o_pb + t->pidt_off[i] * dim * 4, h.pidt_b.data(), (int64_t)h.pidt_b.size());
        std::vector<int32_t> idx;
        idx.assign(h.leaf_level.size(), i);
        put(t->image, t->o_linst + t->leaf_off[i] * 4, idx.data(), (int64_t)idx.size());
        idx.assign(h.pidt_key.size(), i);
        put(t->image, t->o_pinst + t->pidt_off[i] * 4, idx.data(), (int64_t)idx.size());
        idx.assign(h.vtx_lin.size(), i);
        put(t->image, t->o_vinst + t->vtx_off[i] * 4, idx.data(), (int64_t)idx.size());
    }
    put(t->image, t->o_inst, di.data(), ni);
    put(t->image, t->o_vptr, vptr.data(), NV + 1);
    put(t->image, t->o_vinc, vinc.data(), (int64_t)vinc.size());
    put(t->image, t->o_vpptr, vpptr.data(), NV + 1);
    put(t->image, t->o_vpinc, vpinc.data(), (int64_t)vpinc.size());
    put(t->image, t->o_ptab, ptab.data(), (int64_t)ptab.size());
    put(t->image, t->o_ctab, ctab.data(), (int64_t)ctab.size());
    t->reg_kernels = 1;
    for (int i = 0; i < ni; ++i) t->reg_kernels &= di[i].regular && di[i].ptab >= 0;
    t->inst0 = di[0];
    (void)nsten;
    return PIC_OK;
}

void bind(pic_tree *t) {
    char *b = (char *)t->dev;
    DevTree &d = t->dt;
    d.dim = t->dim;
    d.n_inst = t->n_inst;
    d.all_regular = t->all_regular;
    d.n_leaves = t->leaf_off.back();
    d.n_vtx = t->vtx_off.back();
    d.n_pidt = t->pidt_off.back();
    d.n_nodes = t->n_nodes;
    d.inst = (const DevInst *)(b + t->o_inst);
    d.node_child = (const int32_t *)(b + t->o_node);
    d.uni_base = (const uint32_t *)(b + t->o_ubase);
    d.uni_meta = (const uint32_t *)(b + t->o_umeta);
    d.leaf_level = (const uint8_t *)(b + t->o_llev);
    d.leaf_vtx = (const int32_t *)(b + t->o_lvtx);
    d.leaf_pidt = (const int32_t *)(b + t->o_lpidt);
    d.pidt_level = (const uint8_t *)(b + t->o_plev);
    d.leaf_inst = (const int32_t *)(b + t->o_linst);
    d.pidt_inst = (const int32_t *)(b + t->o_pinst);
    d.vtx_inst = (const int32_t *)(b + t->o_vinst);
    d.vinc_ptr = (const int32_t *)(b + t->o_vptr);
    d.vinc = (const int32_t *)(b + t->o_vinc);
    d.vpinc_ptr = (const int32_t *)(b + t->o_vpptr);
    d.vpinc = (const int32_t *)(b + t->o_vpinc);
    d.peano_tab = (const uint32_t *)(b + t->o_ptab);
    d.cell_tab = (const uint32_t *)(b + t->o_ctab);
    d.leaf_coord = (const uint32_t *)(b + t->o_lcoord);
    d.pidt_b = (const uint32_t *)(b + t->o_pb);
    d.status = (uint32_t *)(b + t->o_status);
}

// The FP32 form needs every instance regular with a Peano rank table.
bool valid_precision(const pic_tree *t, int precision) {
    return precision == PIC_F64 || (precision == PIC_F32_OFFSET && t->reg_kernels);
}

bool particles_ok(const pic_tree *t, const pic_particles *p, int precision, bool need_v) {
    if (!p || p->n < 0 || p->n >= (int64_t)INT32_MAX) return false;
    if (p->n == 0) return true;
    for (int k = 0; k < t->dim; ++k) {
        if (precision == PIC_F64 && (!p->x[k] || (need_v && !p->v[k]))) return false;
        if (precision == PIC_F32_OFFSET && (!p->off[k] || (need_v && !p->u[k]))) return false;
    }
    if (t->n_inst > 1 && !p->inst_start_dev) return false;
    return true;
}

}  // namespace

namespace pic {

bool tune_set(Tuning &g, const char *name, int64_t value) {
    if (!name) return false;
    const std::string k(name);
    auto one_of = [value](std::initializer_list<int64_t> ok) {
        for (int64_t v : ok)
            if (v == value) return true;
        return false;
    };
    if (k == "rebin_tile") {
        if (!one_of({2048, 4096})) return false;
        g.rebin_ipt = (int)(value / 256);
    } else if (k == "rebin_radix") {
        if (!one_of({4, 5})) return false;
        g.rebin_radix = (int)value;
    } else if (k == "scatter_mode") {
        if (!one_of({0, 1})) return false;
        g.scatter_mode = (int)value;
    } else if (k == "scatter_group") {
        if (!one_of({1, 2, 4})) return false;
        g.scatter_group = (int)value;
    } else if (k == "deposit_lanes") {
        if (!one_of({0, 16, 32, 64})) return false;
        g.deposit_lanes = (int)value;
    } else if (k == "regular_tables") {
        if (!one_of({0, 1})) return false;
        g.regular_tables = (int)value;
    } else if (k == "step_tile") {
        if (!one_of({0, 1024, 2048, 4096})) return false;
        g.step_ipt = (int)(value / 256);
    } else if (k == "scatter_nt") {
        if (!one_of({0, 1})) return false;
        g.scatter_nt = (int)value;
    } else if (k == "xcd_tiles") {
        if (!one_of({0, 1})) return false;
        g.xcd_tiles = (int)value;
    } else if (k == "deposit_bpw") {
        if (!one_of({1, 2})) return false;
        g.deposit_bpw = (int)value;
    } else if (k == "deposit_batch") {
        if (!one_of({64, 256})) return false;
        g.deposit_batch = (int)value;
    } else if (k == "emit_threads") {
        if (!one_of({512, 1024})) return false;
        g.emit_threads = (int)value;
    } else if (k == "step_fuse") {
        if (!one_of({0, 1, 2})) return false;
        g.step_fuse = (int)value;
    } else if (k == "key_stores") {
        if (!one_of({0, 1, 2})) return false;
        g.key_stores = (int)value;
    } else if (k == "group_match") {
        if (!one_of({0, 1})) return false;
        g.group_match = (int)value;
    } else if (k == "emit_deposit") {
        if (!one_of({0, 1, 2})) return false;
        g.emit_deposit = (int)value;
    } else {
        return false;
    }
    return true;
}

int64_t tune_get(const Tuning &g, const char *name) {
    if (!name) return -1;
    const std::string k(name);
    if (k == "rebin_tile") return 256 * (int64_t)g.rebin_ipt;
    if (k == "rebin_radix") return g.rebin_radix;
    if (k == "scatter_mode") return g.scatter_mode;
    if (k == "scatter_nt") return g.scatter_nt;
    if (k == "scatter_group") return g.scatter_group;
    if (k == "deposit_lanes") return g.deposit_lanes;
    if (k == "step_tile") return 256 * (int64_t)g.step_ipt;
    if (k == "regular_tables") return g.regular_tables;
    if (k == "xcd_tiles") return g.xcd_tiles;
    if (k == "emit_threads") return g.emit_threads;
    if (k == "step_fuse") return g.step_fuse;
    if (k == "emit_deposit") return g.emit_deposit;
    if (k == "group_match") return g.group_match;
    if (k == "key_stores") return g.key_stores;
    if (k == "deposit_bpw") return g.deposit_bpw;
    if (k == "deposit_batch") return g.deposit_batch;
    return -1;
}

}  // namespace pic

extern "C" {

static pic_status tree_create(int32_t dim, int32_t n_inst, const int32_t *max_level, const uint8_t *masks,
                              pic_tree **out) {
    if (!out) return PIC_E_ARG;
    *out = nullptr;
    if ((dim != 2 && dim != 3) || n_inst < 1 || !max_level) return PIC_E_ARG;
    int64_t mask_total = 0;
    for (int i = 0; i < n_inst; ++i) {
        const int L = max_level[i];
        if (L < 0 || L > PIC_MAX_LEVEL || dim * L > 36) return PIC_E_ARG;
        for (int l = 0; l < L; ++l) mask_total += (int64_t)pow3_u64(dim * l);
    }
    if (mask_total > 0 && !masks) return PIC_E_ARG;
    std::unique_ptr<pic_tree> t(new pic_tree());   // freed if a builder throws
    t->dim = dim;
    t->n_inst = n_inst;
    t->tune = g_tune;
    t->inst.resize(n_inst);
    const uint8_t *m = masks;
    for (int i = 0; i < n_inst; ++i) {
        const int L = max_level[i];
        pic_status st = build_instance(dim, L, m, t->inst[i]);
        if (st != PIC_OK) return st;
        for (int l = 0; l < L; ++l) m += pow3_u64(dim * l);
        t->all_regular &= t->inst[i].regular;
        t->max_level = std::max(t->max_level, L);
    }
    pic_status st = assemble(t.get());
    if (st != PIC_OK) return st;
    *out = t.release();
    return PIC_OK;
}

// The host-side builders allocate (tables, masks): no exception leaves the
// C ABI, an exhausted host heap is a status.
pic_status pic_tree_create(int32_t dim, int32_t n_inst, const int32_t *max_level, const uint8_t *masks,
                           pic_tree **out) {
    try {
        return tree_create(dim, n_inst, max_level, masks, out);
    } catch (const std::bad_alloc &) {
        if (out) *out = nullptr;
        return PIC_E_MEMORY;
    }
}

void pic_tree_destroy(pic_tree *tree) { delete tree; }

pic_status pic_tree_get_info(const pic_tree *t, pic_tree_info *info) {
    if (!t || !info) return PIC_E_ARG;
    info->dim = t->dim;
    info->n_inst = t->n_inst;
    info->regular = t->all_regular;
    info->max_level = t->max_level;
    info->n_leaves = t->leaf_off.back();
    info->n_vertices = t->vtx_off.back();
    info->n_pidt = t->pidt_off.back();
    info->n_nodes = t->n_nodes;
    info->device_bytes = t->device_bytes;
    return PIC_OK;
}

pic_status pic_tree_get_instance(const pic_tree *t, int32_t i, pic_instance_info *info) {
    if (!t || !info || i < 0 || i >= t->n_inst) return PIC_E_ARG;
    info->max_level = t->inst[i].L;
    info->regular = t->inst[i].regular;
    info->leaf_offset = t->leaf_off[i];
    info->n_leaves = t->leaf_off[i + 1] - t->leaf_off[i];
    info->vertex_offset = t->vtx_off[i];
    info->n_vertices = t->vtx_off[i + 1] - t->vtx_off[i];
    info->pidt_offset = t->pidt_off[i];
    info->n_pidt = t->pidt_off[i + 1] - t->pidt_off[i];
    return PIC_OK;
}

pic_status pic_tree_leaf_table(const pic_tree *t, uint64_t *key, int32_t *level, int64_t *coord, int32_t *vtx,
                               int32_t *pidt) {
    if (!t) return PIC_E_ARG;
    const int d = t->dim, nc = 1 << d;
    for (int i = 0; i < t->n_inst; ++i) {
        const HostInst &h = t->inst[i];
        const int64_t o = t->leaf_off[i];
        for (size_t r = 0; r < h.leaf_level.size(); ++r) {
            if (key) key[o + r] = h.leaf_key[r];
            if (level) level[o + r] = h.leaf_level[r];
            if (coord) for (int k = 0; k < d; ++k) coord[(o + r) * d + k] = h.leaf_coord[r * d + k];
            for (int c = 0; c < nc; ++c) {
                if (vtx) vtx[(o + r) * nc + c] = h.leaf_vtx[r * nc + c] + (int32_t)t->vtx_off[i];
                if (pidt) pidt[(o + r) * nc + c] = h.leaf_pidt[r * nc + c] + (int32_t)t->pidt_off[i];
            }
        }
    }
    return PIC_OK;
}

pic_status pic_tree_vertex_table(const pic_tree *t, int64_t *pos) {
    if (!t || !pos) return PIC_E_ARG;
    const int d = t->dim;
    for (int i = 0; i < t->n_inst; ++i) {
        const HostInst &h = t->inst[i];
        for (size_t v = 0; v < h.vtx_lin.size(); ++v) {
            int64_t r = h.vtx_lin[v];
            for (int k = 0; k < d; ++k) {
                pos[(t->vtx_off[i] + v) * d + k] = r % h.S;
                r /= h.S;
            }
        }
    }
    return PIC_OK;
}

pic_status pic_tree_pidt_table(const pic_tree *t, uint64_t *pidt_key, int32_t *pidt_level, int64_t *pidt_b) {
    if (!t) return PIC_E_ARG;
    const int d = t->dim;
    for (int i = 0; i < t->n_inst; ++i) {
        const HostInst &h = t->inst[i];
        const int64_t o = t->pidt_off[i];
        for (size_t b = 0; b < h.pidt_key.size(); ++b) {
            if (pidt_key) pidt_key[o + b] = h.pidt_key[b];
            if (pidt_level) pidt_level[o + b] = h.pidt_level[b];
            if (pidt_b) for (int k = 0; k < d; ++k) pidt_b[(o + b) * d + k] = h.pidt_b[b * d + k];
        }
    }
    return PIC_OK;
}

pic_status pic_tree_upload(pic_tree *t, void *buffer, size_t bytes, void *stream) {
    if (!t || !buffer) return PIC_E_ARG;
    if ((int64_t)bytes < t->device_bytes) return PIC_E_CAPACITY;
    if (((uintptr_t)buffer & 255) != 0) return PIC_E_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (hipMemcpyAsync(buffer, t->image.data(), (size_t)t->device_bytes, hipMemcpyHostToDevice, s) != hipSuccess)
        return PIC_E_HIP;
    // the host image must outlive the copy
    if (hipStreamSynchronize(s) != hipSuccess) return PIC_E_HIP;
    t->dev = buffer;
    bind(t);
    return PIC_OK;
}

pic_status pic_status_sync(pic_tree *t, void *stream) {
    if (!t || !t->dev) return PIC_E_STATE;
    hipStream_t s = (hipStream_t)stream;
    uint32_t word = 0;
    if (hipMemcpyAsync(&word, t->dt.status, 4, hipMemcpyDeviceToHost, s) != hipSuccess) return PIC_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return PIC_E_HIP;
    if (launch_status_clear(t, s) != hipSuccess) return PIC_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return PIC_E_HIP;
    if (word & PIC_DEV_NONFINITE) return PIC_E_NONFINITE;
    if (word & PIC_DEV_RANGE) return PIC_E_RANGE;
    return PIC_OK;
}

const char *pic_status_string(pic_status s) {
    switch (s) {
        case PIC_OK: return "ok";
        case PIC_E_ARG: return "invalid argument";
        case PIC_E_SCRATCH: return "scratch buffer too small";
        case PIC_E_CAPACITY: return "buffer too small";
        case PIC_E_NONFINITE: return "non-finite particle coordinate";
        case PIC_E_TREE: return "malformed or oversized tree";
        case PIC_E_HIP: return "HIP runtime error";
        case PIC_E_RANGE: return "coordinate outside the unit box or bin outside the tree";
        case PIC_E_STATE: return "tree not uploaded";
        case PIC_E_MEMORY: return "host memory exhausted";
        default: return "unknown status";
    }
}

pic_status pic_locate(const pic_tree *t, int32_t scheme, int32_t precision, const pic_particles *p,
                      const int64_t *bin_start, uint32_t *bin, void *stream) {
    if (!t || !valid_scheme(scheme) || precision != PIC_F64 || !particles_ok(t, p, precision, false))
        return PIC_E_ARG;
    if (p->n > 0 && !bin) return PIC_E_ARG;
    if (!t->dev) return PIC_E_STATE;
    (void)bin_start;
    return launch_locate(t, scheme, p, bin, (hipStream_t)stream) == hipSuccess ? PIC_OK : PIC_E_HIP;
}

pic_status pic_gather_push(const pic_tree *t, int32_t scheme, int32_t precision, pic_particles *p,
                           const double *const *E, double qmdt, double dt, const pic_push_params *params,
                           const int64_t *bin_start, uint32_t *bin, double *Ep, void *stream) {
    if (!t || !valid_scheme(scheme) || !valid_precision(t, precision) || !particles_ok(t, p, precision, true))
        return PIC_E_ARG;
    if (p->n > 0 && (!E || !bin)) return PIC_E_ARG;
    if (p->n > 0)
        for (int k = 0; k < t->dim; ++k)
            if (!E[k]) return PIC_E_ARG;
    if (precision == PIC_F32_OFFSET && ((p->n > 0 && !bin_start) || Ep)) return PIC_E_ARG;
    if (!t->dev) return PIC_E_STATE;
    hipError_t e = precision == PIC_F64
                       ? launch_gather_push(t, scheme, p, E, qmdt, dt, params, bin, Ep, (hipStream_t)stream)
                       : launch_gather_push_f32(t, scheme, p, E, qmdt, dt, params, bin_start, nullptr, 0, bin,
                                                (hipStream_t)stream);
    return e == hipSuccess ? PIC_OK : PIC_E_HIP;
}

pic_status pic_free_stream(const pic_tree *t, int32_t scheme, int32_t precision, pic_particles *p, double dt,
                           const pic_push_params *params, int32_t boundary, int32_t flops, uint32_t *bin,
                           void *stream) {
    if (!t || !valid_scheme(scheme) || precision != PIC_F64 || !particles_ok(t, p, precision, true))
        return PIC_E_ARG;
    if (boundary != PIC_PERIODIC && boundary != PIC_REFLECTING) return PIC_E_ARG;
    if (flops < 0 || flops > (1 << 20) || (flops & 1)) return PIC_E_ARG;
    if (p->n > 0 && !bin) return PIC_E_ARG;
    if (!t->dev) return PIC_E_STATE;
    return launch_free_stream(t, scheme, p, dt, params ? params->dt_dev : nullptr, boundary, flops, bin,
                              (hipStream_t)stream) == hipSuccess
               ? PIC_OK
               : PIC_E_HIP;
}

pic_status pic_leaf_counts(const pic_tree *t, const pic_particles *p, uint64_t *count, void *stream) {
    if (!t || !particles_ok(t, p, PIC_F64, false) || !count) return PIC_E_ARG;
    if (!t->dev) return PIC_E_STATE;
    return launch_leaf_counts(t, p, (unsigned long long *)count, (hipStream_t)stream) == hipSuccess ? PIC_OK
                                                                                                 : PIC_E_HIP;
}

pic_status pic_vmax(const pic_tree *t, int32_t scheme, const pic_particles *p, const int64_t *bin_start, double dt,
                    double *vmax, uint8_t *quiet, void *scratch, size_t scratch_bytes, void *stream) {
    if (!t || t->n_inst != 1 || !valid_scheme(scheme) || !particles_ok(t, p, PIC_F64, true) || !vmax ||
        !bin_start || !scratch)
        return PIC_E_ARG;
    if (scratch_bytes < vmax_scratch_bytes(t, scheme)) return PIC_E_SCRATCH;
    if (!t->dev) return PIC_E_STATE;
    return launch_vmax(t, scheme, p, bin_start, dt, vmax, quiet, scratch, (hipStream_t)stream) == hipSuccess
               ? PIC_OK
               : PIC_E_HIP;
}

pic_status pic_tree_adapt(const pic_tree *t, const int64_t *leaf_count, int64_t ppc, int32_t max_level,
                          uint8_t *masks, size_t masks_cap, size_t *masks_len, int32_t *new_max_level) {
    if (!t || t->n_inst != 1 || ppc < 0 || !masks_len || !new_max_level) return PIC_E_ARG;
    if (max_level < 0 || max_level > PIC_MAX_LEVEL || t->dim * max_level > 36) return PIC_E_ARG;
    const int64_t nl = (int64_t)t->inst[0].leaf_level.size();
    if (nl > 0 && !leaf_count) return PIC_E_ARG;
    for (int64_t r = 0; r < nl; ++r)
        if (leaf_count[r] < 0) return PIC_E_ARG;
    std::vector<uint8_t> m;
    int L = 0;
    pic_status st;
    try {
        st = adapt_masks(t, leaf_count, ppc, max_level, m, L);
    } catch (const std::bad_alloc &) {
        return PIC_E_MEMORY;
    }
    if (st != PIC_OK) return st;
    *masks_len = m.size();
    *new_max_level = L;
    if (masks_cap < m.size()) return PIC_E_CAPACITY;
    if (!m.empty()) {
        if (!masks) return PIC_E_ARG;
        std::copy(m.begin(), m.end(), masks);
    }
    return PIC_OK;
}

size_t pic_scratch_bytes(const pic_tree *t, int64_t n, int32_t scheme, int32_t precision) {
    if (!t || !valid_scheme(scheme) || n < 0 || !valid_precision(t, precision)) return 0;
    if (precision == PIC_F32_OFFSET) return step_f32_scratch_bytes(t, n, scheme);
    return std::max(rebin_scratch_bytes(t, n, scheme), deposit_scratch_bytes(t, scheme));
}

pic_status pic_rebin(const pic_tree *t, int32_t scheme, int64_t n, const uint32_t *new_bin,
                     const int64_t *old_start, int32_t n_cols, void *const *cols_in, void *const *cols_out,
                     const int32_t *col_bytes, int64_t *new_start, void *scratch, size_t scratch_bytes,
                     pic_rebin_stats *stats, void *stream) {
    if (!t || !valid_scheme(scheme) || n < 0 || n >= (int64_t)INT32_MAX) return PIC_E_ARG;
    if (stats && !old_start) return PIC_E_ARG;
    if (n_cols < 0 || n_cols > 16 || !new_start || !scratch) return PIC_E_ARG;
    if (n > 0 && !new_bin) return PIC_E_ARG;
    if (n_cols > 0 && (!cols_in || !cols_out || !col_bytes)) return PIC_E_ARG;
    Cols c{};
    c.n = n_cols;
    for (int i = 0; i < n_cols; ++i) {
        if (col_bytes[i] != 4 && col_bytes[i] != 8) return PIC_E_ARG;
        if (n > 0 && (!cols_in[i] || !cols_out[i] || cols_in[i] == cols_out[i])) return PIC_E_ARG;
        c.in[i] = cols_in[i];
        c.out[i] = cols_out[i];
        c.bytes[i] = col_bytes[i];
    }
    if (scratch_bytes < rebin_scratch_bytes(t, n, scheme)) return PIC_E_SCRATCH;
    if (!t->dev) return PIC_E_STATE;
    if (stats && launch_rebin_stats(t, scheme, old_start, new_bin, 0, n, stats, (hipStream_t)stream) != hipSuccess)
        return PIC_E_HIP;
    return launch_rebin(t, scheme, n, new_bin, old_start, c, new_start, scratch, scratch_bytes,
                        (hipStream_t)stream) == hipSuccess ? PIC_OK : PIC_E_HIP;
}

pic_status pic_deposit(const pic_tree *t, int32_t scheme, int32_t precision, const pic_particles *p,
                       const int64_t *bin_start, const double *q, double q_uniform, double *rho, void *scratch,
                       size_t scratch_bytes, void *stream) {
    if (!t || !valid_scheme(scheme) || !valid_precision(t, precision) || !particles_ok(t, p, precision, false))
        return PIC_E_ARG;
    if (!bin_start || !rho || !scratch) return PIC_E_ARG;
    if (scratch_bytes < deposit_scratch_bytes(t, scheme)) return PIC_E_SCRATCH;
    if (!t->dev) return PIC_E_STATE;
    hipError_t e = precision == PIC_F64
                       ? launch_deposit(t, scheme, p, bin_start, q, q_uniform, rho, scratch, scratch_bytes,
                                        (hipStream_t)stream)
                       : launch_deposit_f32(t, scheme, p, bin_start, q, q_uniform, rho, scratch, scratch_bytes,
                                            (hipStream_t)stream);
    return e == hipSuccess ? PIC_OK : PIC_E_HIP;
}

pic_status pic_deposit_noalloc(const pic_tree *t, int32_t scheme, int32_t precision, const pic_particles *p,
                               const int64_t *bin_start, const double *q, double q_uniform, double *rho,
                               void *stream) {
    if (!t || !valid_scheme(scheme) || !valid_precision(t, precision) || !particles_ok(t, p, precision, false))
        return PIC_E_ARG;
    if (!bin_start || !rho) return PIC_E_ARG;
    if (deposit_scratch_bytes(t, scheme) > PIC_NOALLOC_SCRATCH_BYTES) return PIC_E_SCRATCH;
    if (!t->dev) return PIC_E_STATE;
    void *scratch = nullptr;
    if (noalloc_scratch(&scratch) != hipSuccess) return PIC_E_HIP;
    ProfSuspend quiet;
    hipError_t e = precision == PIC_F64
                       ? launch_deposit(t, scheme, p, bin_start, q, q_uniform, rho, scratch,
                                        PIC_NOALLOC_SCRATCH_BYTES, (hipStream_t)stream)
                       : launch_deposit_f32(t, scheme, p, bin_start, q, q_uniform, rho, scratch,
                                            PIC_NOALLOC_SCRATCH_BYTES, (hipStream_t)stream);
    return e == hipSuccess ? PIC_OK : PIC_E_HIP;
}

pic_status pic_step(const pic_tree *t, int32_t scheme, int32_t precision, pic_particles *in,
                    const int64_t *bin_start, const double *const *E, double qmdt, double dt,
                    const pic_push_params *params, int32_t n_extra, void *const *extra_in, void *const *extra_out,
                    const int32_t *extra_bytes, int32_t q_column, double q_uniform, pic_particles *out,
                    int64_t *new_bin_start, double *rho, void *scratch, size_t scratch_bytes,
                    pic_rebin_stats *stats, void *stream) {
    if (!t || !valid_scheme(scheme) || !valid_precision(t, precision) || !particles_ok(t, in, precision, true) ||
        !out)
        return PIC_E_ARG;
    if (out->n != in->n || !particles_ok(t, out, precision, true)) return PIC_E_ARG;
    if (in->n > 0 && (!E || !bin_start)) return PIC_E_ARG;
    if (in->n > 0)
        for (int k = 0; k < t->dim; ++k) {
            if (!E[k]) return PIC_E_ARG;
            if (precision == PIC_F64 && (in->x[k] == out->x[k] || in->v[k] == out->v[k])) return PIC_E_ARG;
            if (precision == PIC_F32_OFFSET && (in->off[k] == out->off[k] || in->u[k] == out->u[k]))
                return PIC_E_ARG;
        }
    if (!new_bin_start || !rho || !scratch) return PIC_E_ARG;
    if (n_extra < 0 || n_extra > 16 - 2 * t->dim) return PIC_E_ARG;
    if (n_extra > 0 && (!extra_in || !extra_out || !extra_bytes)) return PIC_E_ARG;
    if (q_column < -1 || q_column >= n_extra) return PIC_E_ARG;
    Cols ex{};
    ex.n = n_extra;
    for (int i = 0; i < n_extra; ++i) {
        if (extra_bytes[i] != 4 && extra_bytes[i] != 8) return PIC_E_ARG;
        if (in->n > 0 && (!extra_in[i] || !extra_out[i] || extra_in[i] == extra_out[i])) return PIC_E_ARG;
        ex.in[i] = extra_in[i];
        ex.out[i] = extra_out[i];
        ex.bytes[i] = extra_bytes[i];
    }
    if (q_column >= 0 && extra_bytes[q_column] != 8) return PIC_E_ARG;
    if (scratch_bytes < pic_scratch_bytes(t, in->n, scheme, precision)) return PIC_E_SCRATCH;
    if (!t->dev) return PIC_E_STATE;
    hipError_t e = precision == PIC_F64
                       ? launch_step(t, scheme, in, bin_start, E, qmdt, dt, params, ex, out, new_bin_start,
                                     q_column, q_uniform, rho, scratch, scratch_bytes, stats, (hipStream_t)stream)
                       : launch_step_f32(t, scheme, in, bin_start, E, qmdt, dt, params, ex, out, new_bin_start,
                                         q_column, q_uniform, rho, scratch, scratch_bytes, stats,
                                         (hipStream_t)stream);
    return e == hipSuccess ? PIC_OK : PIC_E_HIP;
}

pic_status pic_stream_step(const pic_tree *t, int32_t scheme, pic_particles *in, const int64_t *bin_start, double dt,
                           int32_t boundary, int32_t flops, int32_t n_extra, void *const *extra_in,
                           void *const *extra_out, const int32_t *extra_bytes, pic_particles *out,
                           int64_t *new_bin_start, void *scratch, size_t scratch_bytes, pic_rebin_stats *stats,
                           void *stream) {
    if (!t || t->n_inst != 1 || !valid_scheme(scheme) || !particles_ok(t, in, PIC_F64, true) || !out)
        return PIC_E_ARG;
    if (out->n != in->n || !particles_ok(t, out, PIC_F64, true)) return PIC_E_ARG;
    if (boundary != PIC_PERIODIC && boundary != PIC_REFLECTING) return PIC_E_ARG;
    if (flops < 0 || flops > (1 << 20) || (flops & 1)) return PIC_E_ARG;
    if (in->n > 0 && !bin_start) return PIC_E_ARG;
    if (in->n > 0)
        for (int k = 0; k < t->dim; ++k)
            if (in->x[k] == out->x[k] || in->v[k] == out->v[k]) return PIC_E_ARG;
    if (!new_bin_start || !scratch) return PIC_E_ARG;
    if (n_extra < 0 || n_extra > 16 - 2 * t->dim) return PIC_E_ARG;
    if (n_extra > 0 && (!extra_in || !extra_out || !extra_bytes)) return PIC_E_ARG;
    Cols ex{};
    ex.n = n_extra;
    for (int i = 0; i < n_extra; ++i) {
        if (extra_bytes[i] != 4 && extra_bytes[i] != 8) return PIC_E_ARG;
        if (in->n > 0 && (!extra_in[i] || !extra_out[i] || extra_in[i] == extra_out[i])) return PIC_E_ARG;
        ex.in[i] = extra_in[i];
        ex.out[i] = extra_out[i];
        ex.bytes[i] = extra_bytes[i];
    }
    if (scratch_bytes < pic_scratch_bytes(t, in->n, scheme, PIC_F64)) return PIC_E_SCRATCH;
    if (!t->dev) return PIC_E_STATE;
    return launch_stream_step(t, scheme, in, bin_start, dt, boundary, flops, ex, out, new_bin_start, scratch,
                              scratch_bytes, stats, (hipStream_t)stream) == hipSuccess
               ? PIC_OK
               : PIC_E_HIP;
}

pic_status pic_convert(const pic_tree *t, int32_t scheme, int32_t to_precision, pic_particles *p, double dt,
                       const pic_push_params *params, const int64_t *bin_start, uint32_t *bin, void *stream) {
    if (!t || !valid_scheme(scheme) || !t->reg_kernels) return PIC_E_ARG;
    if (to_precision != PIC_F64 && to_precision != PIC_F32_OFFSET) return PIC_E_ARG;
    if (!particles_ok(t, p, PIC_F64, true) || !particles_ok(t, p, PIC_F32_OFFSET, true)) return PIC_E_ARG;
    if (p->n > 0 && to_precision == PIC_F32_OFFSET && !bin) return PIC_E_ARG;
    if (p->n > 0 && to_precision == PIC_F64 && !bin_start) return PIC_E_ARG;
    const bool per_inst = params && params->dt_dev;
    if (!per_inst && !(dt > 0.0)) return PIC_E_ARG;
    if (!t->dev) return PIC_E_STATE;
    return launch_convert(t, scheme, to_precision, p, dt, params, bin_start, bin, (hipStream_t)stream) == hipSuccess
               ? PIC_OK : PIC_E_HIP;
}

pic_status pic_tune_set(const char *name, int64_t value) {
    return tune_set(g_tune, name, value) ? PIC_OK : PIC_E_ARG;
}

int64_t pic_tune_get(const char *name) { return tune_get(g_tune, name); }

pic_status pic_tree_tune_set(pic_tree *t, const char *name, int64_t value) {
    if (!t || !name || std::string(name) == "regular_tables") return PIC_E_ARG;
    return tune_set(t->tune, name, value) ? PIC_OK : PIC_E_ARG;
}

int64_t pic_tree_tune_get(const pic_tree *t, const char *name) {
    if (!t || !name || std::string(name) == "regular_tables") return -1;
    return tune_get(t->tune, name);
}

pic_status pic_stream_push(int32_t dim, int64_t n, double *const *x, double *const *v, double dt, void *stream) {
    if ((dim != 2 && dim != 3) || n < 0 || (n > 0 && (!x || !v))) return PIC_E_ARG;
    for (int k = 0; k < dim && n > 0; ++k)
        if (!x[k] || !v[k]) return PIC_E_ARG;
    return launch_stream_push(dim, n, x, v, dt, (hipStream_t)stream) == hipSuccess ? PIC_OK : PIC_E_HIP;
}

}  // extern "C"
