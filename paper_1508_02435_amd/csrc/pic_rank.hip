// pic_rank.hip -- the middle of the fused step (pic_step): the tile ranking
// of the new keys 2*bin + arrived, the scan of the per-key counts, and the
// placement of every (tile, key) run among the runs of its key.
//
// Ranking inside a round (64 lanes, one slot each) without ordering
// assumptions on LDS atomics: every lane writes its lane id to a per-wave tag
// of its table slot and reads the tag back, which gives all lanes of a slot
// the same representative lane; each lane then ORs its bit into the mask of
// that representative and reads the mask, whose lanes below its own give its
// rank.  The lowest lane of a mask advances the wave's count of the slot.
// The representative a tag ends up with depends on timing, the masks do not.
#include <hip/hip_runtime.h>

#include "pic_launch.h"

namespace pic {

__device__ __forceinline__ uint32_t key_hash(uint32_t k, int bits) { return (k * 0x9E3779B1u) >> (32 - bits); }

template <int HB>
__device__ __forceinline__ uint32_t table_insert(uint32_t *keys, uint32_t k) {
    uint32_t h = key_hash(k, HB);
    for (;;) {
        const uint32_t prev = atomicCAS(&keys[h], 0u, k + 1u);
        if (prev == 0u || prev == k + 1u) return h;
        h = (h + 1u) & ((1u << HB) - 1u);
    }
}

// Slot of key k, or ~0 when absent (at most 2^HB probes).
template <int HB>
__device__ __forceinline__ uint32_t table_find(const uint32_t *keys, uint32_t k) {
    uint32_t h = key_hash(k, HB);
    for (int i = 0; i < (1 << HB); ++i) {
        const uint32_t v = keys[h];
        if (v == k + 1u) return h;
        if (v == 0u) break;
        h = (h + 1u) & ((1u << HB) - 1u);
    }
    return ~0u;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

template <int IPT>
struct RankShape {
    static constexpr int TILE = RB_THREADS * IPT;
    static constexpr int HB = IPT == 4 ? 10 : (IPT == 8 ? 11 : 12);   // TILE table slots
    static constexpr int H = 1 << HB;
    static_assert(H == TILE, "table size");
};

// LDS of the tile ranking.
template <int IPT>
struct alignas(16) RankSmem {
    uint32_t key[RankShape<IPT>::H];            // key + 1 (0: empty); run index after compaction
    uint16_t wc[4][RankShape<IPT>::H];          // per wavefront count of each slot, then its offset
    uint8_t tag[4][RankShape<IPT>::H];          // per wavefront representative lane of each slot
    unsigned long long msk[4][64];              // per wavefront lane mask of each representative
    uint32_t wsum[4];
};

// W consecutive 32-bit LDS words (16-byte aligned for W >= 4, 8-byte for W
// == 2) moved in 16- or 8-byte accesses.
template <int W>
__device__ __forceinline__ void lds_load_words(uint32_t (&r)[W], const uint32_t *p) {
    if constexpr (W % 4 == 0) {
#pragma unroll
        for (int c = 0; c < W / 4; ++c) {
            const uint4 v = ((const uint4 *)p)[c];
            r[4 * c] = v.x; r[4 * c + 1] = v.y; r[4 * c + 2] = v.z; r[4 * c + 3] = v.w;
        }
    } else {
        static_assert(W == 2, "word count");
        const uint2 v = *(const uint2 *)p;
        r[0] = v.x; r[1] = v.y;
    }
}

template <int W>
__device__ __forceinline__ void lds_store_words(uint32_t *p, const uint32_t (&r)[W]) {
    if constexpr (W % 4 == 0) {
#pragma unroll
        for (int c = 0; c < W / 4; ++c) ((uint4 *)p)[c] = make_uint4(r[4 * c], r[4 * c + 1], r[4 * c + 2], r[4 * c + 3]);
    } else {
        static_assert(W == 2, "word count");
        *(uint2 *)p = make_uint2(r[0], r[1]);
    }
}

template <int IPT>
__device__ __forceinline__ void rank_clear(RankSmem<IPT> &S) {
    // the key table and the per-wavefront counts are adjacent: one span of
    // 16-byte stores
    static_assert(offsetof(RankSmem<IPT>, wc) == sizeof(S.key), "layout");
    constexpr int N16 = (int)(sizeof(S.key) + sizeof(S.wc)) / 16;
    const int tid = threadIdx.x;
    uint4 *p = (uint4 *)&S.key[0];
    for (int i = tid; i < N16; i += RB_THREADS) p[i] = make_uint4(0u, 0u, 0u, 0u);
    S.msk[tid >> 6][tid & 63] = 0ull;
}

// Compaction of a ranked tile (the key table holds key + 1 per occupied
// slot, wc[w][slot] the count of wavefront w): in slot order (a block scan)
// every occupied slot gets its run index and tile-local start, written to the
// run table with the key; each run adds (count, 1) to its key's counter and
// lists its address; the per-wavefront counts become per-wavefront offsets
// (counts of the earlier wavefronts) and the key table maps slot -> run
// index.  Called by all threads after a barrier; ends with a barrier.
template <int IPT, typename SM>
__device__ __forceinline__ void tile_compact(SM &S, int64_t tile, int64_t lo, const RebinScratch &sc) {
    const int tid = threadIdx.x;
    // compaction in slot order (a block scan): run index and tile-local
    // start of every occupied slot; the per-wave counts become per-wave
    // offsets (counts of the earlier wavefronts)
    // (a thread's IPT slots are consecutive: their keys and counts move in
    // wide LDS accesses)
    uint32_t k1[IPT], tot[IPT], packed = 0;
    uint32_t cw[4][IPT / 2];
    lds_load_words<IPT>(k1, &S.key[tid * IPT]);
#pragma unroll
    for (int v = 0; v < 4; ++v) lds_load_words<IPT / 2>(cw[v], (const uint32_t *)&S.wc[v][tid * IPT]);
#pragma unroll
    for (int e = 0; e < IPT; ++e) {
        tot[e] = 0;
        const int sh = 16 * (e & 1);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const uint32_t c = (cw[v][e >> 1] >> sh) & 0xffffu;
            cw[v][e >> 1] = (cw[v][e >> 1] & ~(0xffffu << sh)) | (tot[e] << sh);
            tot[e] += c;
        }
        if (k1[e]) packed += 1u + (tot[e] << 16);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) lds_store_words<IPT / 2>((uint32_t *)&S.wc[v][tid * IPT], cw[v]);
    uint32_t total;
    const uint32_t ex = block_excl_scan(packed, S.wsum, &total);
    uint32_t ri = ex & 0xffffu, lb = ex >> 16;
    uint32_t pos[IPT], rr[IPT];
#pragma unroll
    for (int e = 0; e < IPT; ++e) {
        pos[e] = 0u;
        rr[e] = ri;
        if (!k1[e]) continue;
        const uint32_t k = k1[e] - 1u;
        sc.run_key[lo + ri] = k;
        sc.run_info[lo + ri] = lb | (tot[e] << 16);
        // one atomic per run: the key's particle count (high half) and its
        // run count (low half), whose old value is the run's list position;
        // a thread's atomics are all in flight before the first is used
        pos[e] = (uint32_t)atomicAdd((unsigned long long *)&sc.key_cn[k],
                                     ((unsigned long long)tot[e] << 32) | 1ull);
        ++ri;
        lb += tot[e];
    }
    lds_store_words<IPT>(&S.key[tid * IPT], rr);   // slot -> run index
#pragma unroll
    for (int e = 0; e < IPT; ++e) {
        if (!k1[e]) continue;
        const uint32_t k = k1[e] - 1u, a = (uint32_t)lo + rr[e];
        if (pos[e] < sc.klist_cap) sc.klist[(int64_t)k * sc.klist_cap + pos[e]] = a;
        else sc.knext[a] = atomicExch(&sc.khead[k], a + 1u);
    }
    __syncthreads();
    if (tid == 0) sc.tile_nruns[tile] = total & 0xffffu;
}

// Ranks the tile's keys (slot w*64*IPT + j*64 + lane of thread (w, lane),
// ~0 past the end): writes the tile's runs (key, tile-local start | count <<
// 16), adds the per-key counts, and stores run index | rank << 16 for every
// particle.  The table must be cleared and all threads past a barrier.
template <int IPT>
__device__ __forceinline__ void tile_rank(RankSmem<IPT> &S, const uint32_t (&key)[IPT], int64_t tile, int64_t lo,
                                          const RebinScratch &sc, uint32_t *meta) {
    using RS = RankShape<IPT>;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    uint32_t slot[IPT], rk[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        slot[j] = 0u;
        if (key[j] != ~0u) {
            slot[j] = table_find<RS::HB>(S.key, key[j]);
            if (slot[j] == ~0u) slot[j] = table_insert<RS::HB>(S.key, key[j]);
        }
    }
    // wavefront-scope atomic loads and stores: plain LDS accesses that the
    // compiler may neither forward nor reorder against the other lanes' ones
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        rk[j] = 0u;
        if (key[j] == ~0u) continue;
        uint8_t *tg = &S.tag[w][slot[j]];
        uint16_t *cw = &S.wc[w][slot[j]];
        __hip_atomic_store(tg, (uint8_t)lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        const uint32_t rep = __hip_atomic_load(tg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        unsigned long long *mk = &S.msk[w][rep];
        __hip_atomic_fetch_or(mk, 1ull << lane, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        const uint64_t m = __hip_atomic_load(mk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        const uint32_t base = __hip_atomic_load(cw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        const uint32_t below = lanes_below(m);
        if (below == 0u) {
            __hip_atomic_store(cw, (uint16_t)(base + (uint32_t)__popcll(m)), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_WAVEFRONT);
            __hip_atomic_store(mk, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        }
        rk[j] = base + below;
    }
    __syncthreads();
    tile_compact<IPT>(S, tile, lo, sc);
    const int64_t pbase = lo + (int64_t)w * 64 * IPT + lane;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        if (key[j] == ~0u) continue;
        meta[pbase + 64 * j] = S.key[slot[j]] | ((S.wc[w][slot[j]] + rk[j]) << 16);
    }
}

// ------------------------------------------- fused key + ranking, by match
//
// The key pass and the tile ranking in one kernel: a tile of 256 * IPT
// particles per block, wavefront w pushing the slots w*64*IPT + j*64 + lane
// in rounds j (push_one, so the same state and bin as every other pass).
// Inside a round the lanes with equal keys are found by matching: the
// wavefront takes the key of its first unmatched lane, ballots the lanes
// holding it, and repeats until every lane is matched (as many rounds as
// the 64 particles have distinct keys, which sorted input keeps small).
// Only one lane per distinct key (the lowest) touches LDS: it finds or
// inserts the key in the tile's table and advances its wavefront's count of
// it; the others take the table slot and the count from it by a lane
// shuffle, and their rank among the lanes below them from the match mask.
// The ranks follow slot order and do not depend on timing.

template <int IPT>
struct alignas(16) MatchSmem {
    uint32_t key[RankShape<IPT>::H];            // key + 1 (0: empty); run index after compaction
    uint16_t wc[4][RankShape<IPT>::H];          // per wavefront count of each slot, then its offset
    uint32_t wsum[4];
};

template <int IPT>
__device__ __forceinline__ void match_clear(MatchSmem<IPT> &S) {
    static_assert(offsetof(MatchSmem<IPT>, wc) == sizeof(S.key), "layout");
    constexpr int N16 = (int)(sizeof(S.key) + sizeof(S.wc)) / 16;
    uint4 *p = (uint4 *)&S.key[0];
    for (int i = threadIdx.x; i < N16; i += RB_THREADS) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// Rank of this lane's key (~0: no particle) among the wavefront's earlier
// particles with the same key; returns table slot | rank << 16.
template <int IPT>
__device__ __forceinline__ uint32_t match_rank(MatchSmem<IPT> &S, uint32_t key, int w) {
    using RS = RankShape<IPT>;
    const bool live = key != ~0u;
    uint64_t pend = __ballot(live), mine = 0;
    while (pend) {
        const uint32_t k = (uint32_t)__builtin_amdgcn_readlane((int)key, __builtin_ctzll(pend));
        const uint64_t m = __ballot(key == k);
        pend &= ~m;
        if (key == k) mine = m;
    }
    const uint32_t below = lanes_below(mine);
    uint32_t hs = 0u, base = 0u;
    if (live && below == 0u) {
        hs = table_find<RS::HB>(S.key, key);
        if (hs == ~0u) hs = table_insert<RS::HB>(S.key, key);
        base = S.wc[w][hs];
        S.wc[w][hs] = (uint16_t)(base + (uint32_t)__popcll(mine));
    }
    const int leader = live ? __builtin_ctzll(mine) : (int)__lane_id();
    hs = (uint32_t)__shfl((int)hs, leader, 64);
    base = (uint32_t)__shfl((int)base, leader, 64);
    return live ? (hs | ((base + below) << 16)) : ~0u;
}

template <int D, int SCHEME, bool REG, bool MULTI, int IPT>
__global__ __launch_bounds__(RB_THREADS) void k_step_keyrank(DevTree t, DevInst in0, F64Ptrs P, int64_t n,
                                                            double qmdt0, double dt0, const double *qa,
                                                            const double *da, const int64_t *inst_start,
                                                            const int64_t *old_start, uint32_t n_bins,
                                                            RebinScratch sc, uint32_t *keys_out) {
    using RS = RankShape<IPT>;
    __shared__ MatchSmem<IPT> S;
    __shared__ int32_t lds[REG ? 1 : PIC_LDS_NODES];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t tile = blockIdx.x;
    const int64_t lo = tile * RS::TILE;
    match_clear<IPT>(S);
    const int lds_n = MULTI ? 0 : stage_nodes<REG>(t, in0, lds);
    __syncthreads();   // table cleared
    const int64_t pbase = lo + (int64_t)w * 64 * IPT + lane;
    uint32_t bad = 0;
    // the next round's state is loaded while this round is pushed and ranked
    double xn[D], vn[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        xn[k] = pbase < n ? P.x[k][pbase] : 0.0;
        vn[k] = pbase < n ? P.v[k][pbase] : 0.0;
    }
    uint32_t res[IPT];   // per particle: table slot | rank << 16
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int64_t p = pbase + 64 * j;
        double xv[D], vv[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            xv[k] = xn[k];
            vv[k] = vn[k];
        }
        if (j + 1 < IPT && p + 64 < n) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                xn[k] = P.x[k][p + 64];
                vn[k] = P.v[k][p + 64];
            }
        }
        uint32_t key = ~0u;
        if (p < n) {
            key = step_key_one<D, SCHEME, REG, MULTI>(t, in0, P, p, xv, vv, qmdt0, dt0, qa, da, inst_start,
                                                      old_start, n_bins, lds, lds_n, bad);
            if (keys_out) keys_out[p] = key;
        }
        res[j] = match_rank<IPT>(S, key, w);
    }
    if (bad) flag_status(t.status, bad);
    __syncthreads();
    tile_compact<IPT>(S, tile, lo, sc);
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint32_t r = res[j];
        if (r == ~0u) continue;
        const uint32_t hs = r & 0xffffu;
        sc.meta[pbase + 64 * j] = S.key[hs] | (((uint32_t)S.wc[w][hs] + (r >> 16)) << 16);
    }
}

// Group pass: ranks the keys the key pass wrote, one tile of 256 * IPT
// particles per block (tile_rank).
template <int IPT>
__global__ __launch_bounds__(RB_THREADS) void k_step_group(const uint32_t *keys, int64_t n, RebinScratch sc,
                                                          uint32_t *meta, int xcd) {
    using RS = RankShape<IPT>;
    __shared__ RankSmem<IPT> S;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x, xcd);
    const int64_t lo = tile * RS::TILE;
    rank_clear<IPT>(S);
    const int64_t base = lo + (int64_t)w * 64 * IPT + lane;
    uint32_t key[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) key[j] = base + 64 * j < n ? keys[base + 64 * j] : ~0u;
    __syncthreads();   // table cleared
    tile_rank<IPT>(S, key, tile, lo, sc, meta);
}

// Group pass by matching: the same ranks as k_step_group (slot order), with
// one LDS access per distinct key of a wavefront round instead of several per
// particle (match_rank).
template <int IPT>
__global__ __launch_bounds__(RB_THREADS) void k_step_group_match(const uint32_t *keys, int64_t n, RebinScratch sc,
                                                                uint32_t *meta, int xcd) {
    using RS = RankShape<IPT>;
    __shared__ MatchSmem<IPT> S;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x, xcd);
    const int64_t lo = tile * RS::TILE;
    match_clear<IPT>(S);
    const int64_t base = lo + (int64_t)w * 64 * IPT + lane;
    uint32_t key[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) key[j] = base + 64 * j < n ? keys[base + 64 * j] : ~0u;
    __syncthreads();   // table cleared
    uint32_t res[IPT];   // per particle: table slot | rank << 16
#pragma unroll
    for (int j = 0; j < IPT; ++j) res[j] = match_rank<IPT>(S, key[j], w);
    __syncthreads();
    tile_compact<IPT>(S, tile, lo, sc);
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const uint32_t r = res[j];
        if (r == ~0u) continue;
        const uint32_t hs = r & 0xffffu;
        meta[base + 64 * j] = S.key[hs] | (((uint32_t)S.wc[w][hs] + (r >> 16)) << 16);
    }
}

// Fused step, middle.  Scan: each block of SP_THREADS threads scans the
// (count, runs) pairs of SP_KEYS keys; its first wavefront publishes the
// block's aggregate and looks back over up to 64 predecessors at a time (one
// lane per predecessor) for the exclusive prefix.  Place: per key, its runs
// (the direct list the ranking filled, then for keys with more than klist_cap
// runs the linked rest) sorted by run address, i.e. tile order, and given
// their destinations.

__global__ __launch_bounds__(SP_THREADS) void k_step_scan(uint32_t n_keys, uint32_t n_bins, int64_t n, RebinScratch sc,
                                                          int64_t *new_start, uint32_t *status) {
    // A block's position in the scan comes from a ticket taken when it
    // starts, so every predecessor it waits for has started before it (the
    // wait is bounded all the same).  The ticket counter is cleared by the
    // pass that clears the per-key counters.
    __shared__ uint32_t s_wsum[4];
    __shared__ uint64_t s_excl;
    __shared__ uint32_t s_bid;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) s_bid = atomicAdd(sc.scan_ctr, 1u);
    __syncthreads();
    const uint32_t bid = s_bid;
    const uint64_t k0 = (uint64_t)bid * SP_KEYS + (uint64_t)tid * SP_KPT;
    uint32_t c[SP_KPT], r[SP_KPT];
    uint32_t cs = 0, rs = 0;
#pragma unroll
    for (int j = 0; j < SP_KPT; ++j) {
        const uint64_t k = k0 + j;
        c[j] = r[j] = 0;
        if (k < n_keys) {
            const uint64_t cn = sc.key_cn[k];
            c[j] = (uint32_t)(cn >> 32);
            r[j] = (uint32_t)cn;
        }
        cs += c[j];
        rs += r[j];
    }
    uint32_t ctot, rtot;
    const uint32_t cex = block_excl_scan(cs, s_wsum, &ctot);
    const uint32_t rex = block_excl_scan(rs, s_wsum, &rtot);
    // look-back: every thread reads one of the 256 predecessors before the
    // window start; the nearest published prefix ends the walk
    __shared__ uint64_t s_pc[4], s_pr[4];
    __shared__ int s_stop[4];
    __shared__ uint32_t s_done, s_fail;
    const uint64_t agg = ((uint64_t)ctot << 31) | rtot;
    if (tid == 0) {
        __hip_atomic_store(&sc.scan_state[bid], (bid == 0 ? ST_PRE : ST_AGG) | agg, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        s_done = bid == 0 ? 1u : 0u;
        s_fail = 0u;
    }
    uint64_t ec = 0, er = 0;
    __syncthreads();
    for (int64_t j0 = (int64_t)bid - 1; !s_done; j0 -= SP_THREADS) {
        const int64_t j = j0 - tid;
        uint64_t st = ST_PRE;   // before block 0: an empty prefix
        if (j >= 0) {
            uint32_t spins = 0;
            for (;;) {
                st = __hip_atomic_load(&sc.scan_state[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((st >> 62) != 0) break;
                if (++spins > (1u << 22)) {   // bounded wait: report instead of hanging
                    s_fail = 1u;
                    st = ST_PRE;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        // nearest published prefix: the smallest thread index with a PRE flag
        const uint64_t pre = __ballot((st >> 62) == 2);
        if (lane == 0) s_stop[w] = pre ? 64 * w + __builtin_ctzll(pre) : SP_THREADS;
        __syncthreads();
        int stop = SP_THREADS;
#pragma unroll
        for (int v = 0; v < 4; ++v) stop = min(stop, s_stop[v]);
        uint64_t vc = tid <= stop ? ((st & ST_VAL) >> 31) : 0, vr = tid <= stop ? (st & 0x7fffffffull) : 0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            vc += (uint64_t)__shfl_xor((long long)vc, o, 64);
            vr += (uint64_t)__shfl_xor((long long)vr, o, 64);
        }
        if (lane == 0) {
            s_pc[w] = vc;
            s_pr[w] = vr;
        }
        __syncthreads();
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            ec += s_pc[v];
            er += s_pr[v];
        }
        if (tid == 0 && (stop < SP_THREADS || j0 - SP_THREADS < 0)) s_done = 1u;
        __syncthreads();
    }
    if (tid == 0) {
        if (s_fail) atomicOr(status, PIC_DEV_RANGE);
        s_excl = ((ec & 0x7fffffffull) << 31) | (er & 0x7fffffffull);
        if (bid != 0)
            __hip_atomic_store(&sc.scan_state[bid],
                               ST_PRE | (((ec + ctot) & 0x7fffffffull) << 31) | ((er + rtot) & 0x7fffffffull),
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    uint32_t cb = (uint32_t)(s_excl >> 31) + cex, rb = (uint32_t)(s_excl & 0x7fffffffull) + rex;
#pragma unroll
    for (int j = 0; j < SP_KPT; ++j) {
        const uint64_t k = k0 + j;
        if (k < n_keys) {
            sc.key_base[k] = cb;
            sc.list_off[k] = rb;
            if ((k & 1) == 0) new_start[k >> 1] = cb;
            if (k + 1 == n_keys) {
                sc.list_off[n_keys] = rb + r[j];
                new_start[n_bins] = n;
            }
        }
        cb += c[j];
        rb += r[j];
    }
}

// Destinations of a key's 65..128 runs, two per lane: each run's
// destination is the key base plus the counts of the runs with smaller
// addresses, found by comparing against every run of the key in turn.
__device__ __forceinline__ void place_counted(const RebinScratch &sc, const uint32_t *lst, uint32_t l0, uint32_t len,
                                              uint32_t kb, int lane, uint32_t pos0) {
    uint32_t a0 = ~0u, c0 = 0u, a1 = ~0u, c1 = 0u;
    if ((uint32_t)lane < len) {
        a0 = lst[l0 + lane];
        c0 = sc.run_info[a0] >> 16;
    }
    if ((uint32_t)lane + 64u < len) {
        a1 = lst[l0 + 64 + lane];
        c1 = sc.run_info[a1] >> 16;
    }
    uint32_t b0 = 0u, b1 = 0u, r0 = 0u, r1 = 0u;
    for (int j = 0; j < 64; ++j) {
        const uint32_t x0 = (uint32_t)__builtin_amdgcn_readlane((int)a0, j);
        const uint32_t y0 = (uint32_t)__builtin_amdgcn_readlane((int)c0, j);
        const uint32_t x1 = (uint32_t)__builtin_amdgcn_readlane((int)a1, j);
        const uint32_t y1 = (uint32_t)__builtin_amdgcn_readlane((int)c1, j);
        b0 += (x0 < a0 ? y0 : 0u) + (x1 < a0 ? y1 : 0u);
        b1 += (x0 < a1 ? y0 : 0u) + (x1 < a1 ? y1 : 0u);
        r0 += (x0 < a0 ? 1u : 0u) + (x1 < a0 ? 1u : 0u);
        r1 += (x0 < a1 ? 1u : 0u) + (x1 < a1 ? 1u : 0u);
    }
    if ((uint32_t)lane < len) {
        sc.run_dest[a0] = kb + b0;
        sc.run_pos[a0] = pos0 + r0;
    }
    if ((uint32_t)lane + 64u < len) {
        sc.run_dest[a1] = kb + b1;
        sc.run_pos[a1] = pos0 + r1;
    }
}

#ifndef PIC_PLACE_KW
#define PIC_PLACE_KW 8
#endif

template <int KW>
__global__ __launch_bounds__(256) void k_step_place(RebinScratch sc, uint32_t n_keys) {
    // Besides its destination every run gets its position among all runs
    // sorted by (key, tile): the key's list offset plus its rank among the
    // key's runs by address (tile order).  A wavefront takes 64 / KW keys at
    // a time, KW lanes each; keys with up to 16 runs then take 16 lanes, four
    // at a time, and longer ones the whole wavefront in turn.
    static_assert(KW == 8 || KW == 16, "lanes per key");
    constexpr int NG = 64 / KW;
    const int lane = threadIdx.x & 63;
    const int grp = lane / KW, sub = lane % KW;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t k0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * NG; k0 < n_keys;
         k0 += waves * NG) {
        const int64_t key = k0 + grp;
        uint32_t len = 0, kb = 0, lo = 0;
        if (key < n_keys) {
            len = (uint32_t)sc.key_cn[key];
            kb = sc.key_base[key];
            lo = sc.list_off[key];
        }
        if (__ballot(len != 0u) == 0) continue;   // all NG keys empty
        const uint32_t cap = sc.klist_cap;        // >= 16
        if (len <= (uint32_t)KW) place_sorted<KW>(sc, sc.klist, (uint32_t)(key * cap), len, kb, sub, sc.run_pos, lo);
        if (KW < 16) {
            // keys with KW+1..16 runs: four at a time, 16 lanes each (the
            // h-th such key, by lane, goes to lane group h)
            uint64_t mid = __ballot(sub == 0 && len > (uint32_t)KW && len <= 16u);
            const int h = lane >> 4, s16 = lane & 15;
            while (mid) {
                uint64_t m = mid;
                for (int i = 0; i < h && m; ++i) m &= m - 1;
                const int src = m ? __builtin_ctzll(m) : 0;
                const uint32_t mlen = (uint32_t)__shfl((int)len, src, 64);
                const uint32_t mkb = (uint32_t)__shfl((int)kb, src, 64);
                const uint32_t mlo = (uint32_t)__shfl((int)lo, src, 64);
                const int64_t mk = k0 + src / KW;
                place_sorted<16>(sc, sc.klist, (uint32_t)(mk * cap), m ? mlen : 0u, mkb, s16, sc.run_pos, mlo);
                for (int i = 0; i < 4 && mid; ++i) mid &= mid - 1;
            }
        }
        for (int g = 0; g < NG; ++g) {
            const int64_t gk = k0 + g;
            const uint32_t glen = (uint32_t)__shfl((int)len, g * KW, 64);
            const uint32_t gkb = (uint32_t)__shfl((int)kb, g * KW, 64);
            const uint32_t glo = (uint32_t)__shfl((int)lo, g * KW, 64);
            if (glen <= (uint32_t)(KW < 16 ? 16 : KW)) continue;
            if (glen <= 64u && glen <= cap) {
                place_sorted<64>(sc, sc.klist, (uint32_t)(gk * cap), glen, gkb, lane, sc.run_pos, glo);
                continue;
            }
            if (glen <= cap) {
                place_counted(sc, sc.klist, (uint32_t)(gk * cap), glen, gkb, lane, glo);
                continue;
            }
            // a long list: gathered into its exact slot range of the list
            // array (direct part by the lanes, linked part by lane 0), then
            // every run counts the runs before it
            const uint32_t l0 = glo;
            for (uint32_t i = lane; i < cap; i += 64) sc.list[l0 + i] = sc.klist[gk * cap + i];
            if (lane == 0) {
                uint32_t q = cap;
                for (uint32_t e = sc.khead[gk]; e != 0u && q < glen; e = sc.knext[e - 1u]) sc.list[l0 + q++] = e - 1u;
            }
            __threadfence();   // lane 0's entries visible to the other lanes' loads
            for (uint32_t q = lane; q < glen; q += 64) {
                const uint32_t a = sc.list[l0 + q];
                uint32_t before = 0, rank = 0;
                for (uint32_t j = l0; j < l0 + glen; ++j) {
                    const uint32_t bb = sc.list[j];
                    if (bb < a) {
                        before += sc.run_info[bb] >> 16;
                        ++rank;
                    }
                }
                sc.run_dest[a] = gkb + before;
                sc.run_pos[a] = l0 + rank;
            }
        }
    }
}

// ----------------------------------------------------------------- launchers

void launch_keyrank(const pic_tree *t, int scheme, const F64Ptrs &P, int64_t n, double qmdt, double dt,
                    const double *qa, const double *da, const int64_t *inst_start, const int64_t *old_start,
                    uint32_t n_bins, int tile, const RebinScratch &sc, uint32_t *keys_out, hipStream_t s) {
    if (n == 0) return;
    const dim3 g((unsigned)((n + tile - 1) / tile)), b(RB_THREADS);
#define PIC_KR(D, SCH, REG, MULTI, IPT)                                                                      \
    PIC_LAUNCH("step_keyrank", (k_step_keyrank<D, SCH, REG, MULTI, IPT>), g, b, 0, s, t->dt, t->inst0, P, n, qmdt, \
               dt, qa, da, inst_start, old_start, n_bins, sc, keys_out)
#define PIC_KR_T(D, SCH, REG, MULTI)                                                                         \
    do {                                                                                                     \
        if (tile == 1024) PIC_KR(D, SCH, REG, MULTI, 4); else PIC_KR(D, SCH, REG, MULTI, 8);                \
    } while (0)
#define PIC_KR_RM(D, SCH)                                                                                    \
    do {                                                                                                     \
        const bool multi = t->n_inst > 1, reg = t->reg_kernels != 0;                                         \
        if (multi) { if (reg) PIC_KR_T(D, SCH, true, true); else PIC_KR_T(D, SCH, false, true); }            \
        else { if (reg) PIC_KR_T(D, SCH, true, false); else PIC_KR_T(D, SCH, false, false); }                \
    } while (0)
    if (t->dim == 2) {
        if (scheme == PIC_PIT) PIC_KR_RM(2, 0); else PIC_KR_RM(2, 1);
    } else {
        if (scheme == PIC_PIT) PIC_KR_RM(3, 0); else PIC_KR_RM(3, 1);
    }
#undef PIC_KR_RM
#undef PIC_KR_T
#undef PIC_KR
}

void launch_group(const uint32_t *keys, int64_t n, int tile, bool match, const RebinScratch &sc, hipStream_t s) {
    const int64_t tiles = (n + tile - 1) / tile;
    if (n == 0) return;
    if (match) {
        if (tile == 1024)
            PIC_LAUNCH("step_group", (k_step_group_match<4>), dim3(tiles), dim3(RB_THREADS), 0, s, keys, n, sc, sc.meta,
                       0);
        else if (tile == 4096)
            PIC_LAUNCH("step_group", (k_step_group_match<16>), dim3(tiles), dim3(RB_THREADS), 0, s, keys, n, sc,
                       sc.meta, 0);
        else
            PIC_LAUNCH("step_group", (k_step_group_match<8>), dim3(tiles), dim3(RB_THREADS), 0, s, keys, n, sc, sc.meta,
                       0);
    } else if (tile == 1024) {
        PIC_LAUNCH("step_group", (k_step_group<4>), dim3(tiles), dim3(RB_THREADS), 0, s, keys, n, sc, sc.meta, 0);
    } else if (tile == 4096) {
        PIC_LAUNCH("step_group", (k_step_group<16>), dim3(tiles), dim3(RB_THREADS), 0, s, keys, n, sc, sc.meta, 0);
    } else {
        PIC_LAUNCH("step_group", (k_step_group<8>), dim3(tiles), dim3(RB_THREADS), 0, s, keys, n, sc, sc.meta, 0);
    }
}

// The middle of the fused step: scan, then placement from the per-key lists.
void launch_step_middle(const pic_tree *t, int64_t n, int64_t n_bins, const RebinScratch &sc,
                               int64_t *new_start, hipStream_t s) {
    const int64_t keys = 2 * n_bins;
    PIC_LAUNCH("step_scan", k_step_scan, dim3((keys + SP_KEYS - 1) / SP_KEYS), dim3(SP_THREADS), 0, s, (uint32_t)keys,
               (uint32_t)n_bins, n, sc, new_start, t->dt.status);
    if (n > 0)
        PIC_LAUNCH("step_place", k_step_place<PIC_PLACE_KW>, dim3(grid_for(keys, 64 / PIC_PLACE_KW * 4, 1 << 16)),
                   dim3(256), 0, s, sc, (uint32_t)keys);
}

}  // namespace pic
