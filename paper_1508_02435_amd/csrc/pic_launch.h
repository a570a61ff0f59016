// pic_launch.h -- host-side helpers shared by the launchers of the kernel
// sources: grid sizes, pointer bundles, the scratch layout, and the
// launchers one source exports to another.
#pragma once

#include "pic_device.h"

namespace pic {

inline int grid_for(int64_t items, int per_block, int cap) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

inline F64Ptrs make_ptrs(const pic_tree *t, const pic_particles *p, const double *const *E, double *Ep) {
    F64Ptrs P{};
    for (int k = 0; k < 3; ++k) {
        P.x[k] = p->x[k];
        P.v[k] = p->v[k];
        P.E[k] = E ? E[k] : nullptr;
        P.Ep[k] = Ep ? Ep + (int64_t)k * p->n : nullptr;
    }
    (void)t;
    return P;
}

inline int64_t n_bins_of(const pic_tree *t, int scheme) {
    return scheme == PIC_PIT ? t->leaf_off.back() : t->pidt_off.back();
}

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct RebinLayout {
    size_t tile_bin, perm, run_key, run_info, run_dest, tile_nruns, key_cnt, key_nruns, key_fill, key_cn, key_base,
        list_off,
        list, scan_state, scan_ctr, khead, run_wcnt, meta, keys, klist, knext, wave_bin, run_pos, run_part, bin_part,
        total;
    uint32_t klist_cap;
};

// run_ns: doubles of each run's deposit partial when the writing pass of the
// fused step deposits (0 otherwise).
inline RebinLayout rebin_layout(int64_t n, int64_t n_bins, int tile, int run_ns = 0) {
    RebinLayout L{};
    const int64_t tiles = (n + tile - 1) / tile;
    const int64_t slots = tiles * tile;
    const int64_t keys = 2 * n_bins;
    const int64_t scan_blocks = (keys + std::min(SP_KEYS, SCAN_TILE) - 1) / std::min(SP_KEYS, SCAN_TILE);
    size_t o = 0;
    L.tile_bin = o; o = align256(o + tiles * 8);
    L.perm = o; o = align256(o + slots * 2);
    L.run_key = o; o = align256(o + slots * 4);
    L.run_info = o; o = align256(o + slots * 4);
    L.run_dest = o; o = align256(o + slots * 4);
    L.tile_nruns = o; o = align256(o + tiles * 4);
    L.key_cnt = o; o = align256(o + keys * 4);      // key_cnt, key_nruns, key_fill, the scan state and
    L.key_nruns = o; o = align256(o + keys * 4);    // the block counter are contiguous: one fill clears
    L.key_fill = o; o = align256(o + keys * 4);     // them all
    L.key_cn = o; o = align256(o + keys * 8);
    L.scan_state = o; o = align256(o + scan_blocks * 8);
    L.scan_ctr = o; o = align256(o + 4);
    L.khead = o; o = align256(o + keys * 4);
    L.key_base = o; o = align256(o + keys * 4);
    L.list_off = o; o = align256(o + (keys + 1) * 4);
    L.list = o; o = align256(o + slots * 4);
    L.run_wcnt = o; o = align256(o + slots * 8);
    L.meta = o; o = align256(o + slots * 4);
    L.keys = o; o = align256(o + slots * 4);
    // the direct run list of a key: four times the slots per key, rounded up
    // to a power of two, between 16 and KLIST_CAP (a denser key spills into
    // the linked rest)
    uint32_t cap = 16;
    while (cap < (uint32_t)KLIST_CAP && (int64_t)cap * keys < 4 * slots) cap *= 2;
    L.klist_cap = cap;
    L.klist = o; o = align256(o + keys * (int64_t)cap * 4);
    L.knext = o; o = align256(o + slots * 4);
    L.wave_bin = o; o = align256(o + (slots / 64 + 1) * 4);
    L.run_pos = o; o = align256(o + slots * 4);
    L.run_part = o; o = align256(o + slots * 8 * run_ns);
    L.bin_part = o; o = align256(o + n_bins * 8 * run_ns);
    L.total = o;
    return L;
}

inline RebinScratch bind_scratch(const RebinLayout &L, char *base) {
    RebinScratch sc;
    sc.tile_bin = (uint32_t *)(base + L.tile_bin);
    sc.perm = (uint16_t *)(base + L.perm);
    sc.run_key = (uint32_t *)(base + L.run_key);
    sc.run_info = (uint32_t *)(base + L.run_info);
    sc.run_dest = (uint32_t *)(base + L.run_dest);
    sc.tile_nruns = (uint32_t *)(base + L.tile_nruns);
    sc.key_cnt = (uint32_t *)(base + L.key_cnt);
    sc.key_nruns = (uint32_t *)(base + L.key_nruns);
    sc.key_cn = (uint64_t *)(base + L.key_cn);
    sc.key_fill = (uint32_t *)(base + L.key_fill);
    sc.key_base = (uint32_t *)(base + L.key_base);
    sc.list_off = (uint32_t *)(base + L.list_off);
    sc.list = (uint32_t *)(base + L.list);
    sc.scan_state = (uint64_t *)(base + L.scan_state);
    sc.scan_ctr = (uint32_t *)(base + L.scan_ctr);
    sc.run_wcnt = (uint64_t *)(base + L.run_wcnt);
    sc.meta = (uint32_t *)(base + L.meta);
    sc.keys = (uint32_t *)(base + L.keys);
    sc.klist = (uint32_t *)(base + L.klist);
    sc.khead = (uint32_t *)(base + L.khead);
    sc.knext = (uint32_t *)(base + L.knext);
    sc.wave_bin = (uint32_t *)(base + L.wave_bin);
    sc.run_pos = (uint32_t *)(base + L.run_pos);
    sc.run_part = (double *)(base + L.run_part);
    sc.klist_cap = L.klist_cap;
    return sc;
}

// Clears the per-call counters (`n_zero` words from `zero`) and, when
// `old_start` is given, fills the per-tile old-bin bounds and the old bin of
// every 64th slot (pic_rebin.hip).
void launch_prep(uint32_t *zero, int64_t n_zero, const int64_t *old_start, int64_t n_bins, int64_t n, int tile,
                 const RebinScratch &sc, hipStream_t s);
// The fused step's key pass and tile ranking in one kernel (pic_rank.hip);
// keys_out (nullable) receives every particle's key as well.
void launch_keyrank(const pic_tree *t, int scheme, const F64Ptrs &P, int64_t n, double qmdt, double dt,
                    const double *qa, const double *da, const int64_t *inst_start, const int64_t *old_start,
                    uint32_t n_bins, int tile, const RebinScratch &sc, uint32_t *keys_out, hipStream_t s);
// The tile ranking of the fused step over keys in memory (pic_rank.hip).
void launch_group(const uint32_t *keys, int64_t n, int tile, bool match, const RebinScratch &sc, hipStream_t s);
// Per-vertex sums of the deposit's per-bin partials (pic_kernels.hip); `reg`
// selects the arithmetic enumeration of regular trees.
void launch_deposit_vertices(const pic_tree *t, int scheme, bool reg, const double *partial, bool use_q,
                             double q_uniform, double *rho, hipStream_t s);
// Scan of the per-key (count, runs) pairs and run placement (pic_rank.hip).
void launch_step_middle(const pic_tree *t, int64_t n, int64_t n_bins, const RebinScratch &sc, int64_t *new_start,
                        hipStream_t s);

}  // namespace pic
