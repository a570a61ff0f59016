// pic_rebin.hip -- the stable re-bin of pic_rebin: a stable counting sort by
// bin that moves every particle record exactly once: (1) per tile of 2048 or
// 4096 particles an LDS radix sort of the tile's bins with a stayer/arrival
// flag, emitting runs; (2) one decoupled-lookback scan over all (bin, flag)
// keys; (3) per-key run lists give each run its place among the runs of the
// same key in tile order; (4) an LDS-staged scatter writes each run
// contiguously.  Atomics touch integer counters only, and every output
// position is independent of scheduling.
#include <hip/hip_runtime.h>

#include "pic_launch.h"

namespace pic {

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Counter layout of the LDS radix passes: digit-major index f = d*256 + t,
// padded by one word every 32 so that both the per-thread column accesses of
// the counting phase and the per-thread row segments of the scan phase fall
// into distinct banks.
__device__ __forceinline__ int cpad(int f) { return f + (f >> 5); }

// Pass 1: per tile, a stable LDS radix sort of the particle slots groups them
// into runs of equal key 2*bin + arrived.  IPT slots per thread, RADIX bits
// per pass.  Each thread counts the digits of its own slots in registers
// (8-bit counters packed in 64-bit words), so a pass costs a few independent
// LDS round trips instead of a read-modify-write chain per slot.
template <int IPT, int RADIX, bool STAGE>
struct TileSmem {
    static constexpr int TILE = RB_THREADS * IPT;
    static constexpr int DIG = 1 << RADIX;
    static constexpr int NCNT_PAD = DIG * RB_THREADS + DIG * RB_THREADS / 32 + 1;
    // the counter area doubles as run-start table and, with STAGE, as an
    // 8-byte staging buffer for one column of the tile
    static constexpr int NSCR = (STAGE && 2 * TILE > NCNT_PAD) ? 2 * TILE : (NCNT_PAD > TILE + 1 ? NCNT_PAD : TILE + 1);
    uint32_t key[TILE];
    uint16_t item[2][TILE];
    uint32_t cnt[NSCR];
    uint32_t wsum[4];
    uint32_t misc[4];
};

// On entry S.key[i] holds the new bin of tile slot i (i < cnt) and all
// threads have passed a barrier.  Sorts the slots by (bin, arrived), writes
// the tile's run table and key counts, and returns the item buffer that
// holds the sorted order (sorted slot -> tile slot).  S.cnt holds the run
// starts afterwards (n_runs + 1 entries).
template <int IPT, int RADIX, bool STAGE>
__device__ int tile_sort_emit(TileSmem<IPT, RADIX, STAGE> &S, const int64_t *old_start, int64_t tile, int cnt,
                              uint32_t n_bins, RebinScratch &sc, uint32_t *status, uint32_t &n_runs_out) {
    constexpr int TILE = RB_THREADS * IPT;
    constexpr int DIG = 1 << RADIX;
    const int tid = threadIdx.x;
    const int64_t lo = tile * TILE;
    uint32_t nbv[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int i = tid * IPT + j;
        uint32_t nb = i < cnt ? S.key[i] : 0u;
        if (i < cnt && nb >= n_bins) {
            flag_status(status, PIC_DEV_RANGE);
            nb = n_bins - 1;
        }
        nbv[j] = nb;
    }
    __syncthreads();

    // old bin of each slot: the segment of old_start that holds it
    if (old_start) {
        for (int i = tid; i < TILE; i += RB_THREADS) S.cnt[i] = 0;  // head counts
        // b0: the bin holding slot 0; bins in (b0, b1) start inside the tile
        if (tid == 0) {
            S.misc[0] = min(sc.tile_bin[2 * tile], n_bins - 1);
            S.misc[1] = min(sc.tile_bin[2 * tile + 1], n_bins);
        }
        __syncthreads();
        const uint32_t b0 = S.misc[0], b1 = S.misc[1];
        for (uint32_t b = b0 + 1 + tid; b < b1; b += RB_THREADS) {
            const int64_t at = old_start[b] - lo;
            if (at >= 0 && at < cnt) atomicAdd(&S.cnt[(int)at], 1u);
        }
        __syncthreads();
        // inclusive scan of head counts: slot i lies in bin b0 + heads(<= i)
        uint32_t loc[IPT];
        uint32_t sum = 0;
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            sum += S.cnt[tid * IPT + j];
            loc[j] = sum;
        }
        uint32_t tot;
        uint32_t base = block_excl_scan(sum, S.wsum, &tot);
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const int i = tid * IPT + j;
            if (i < cnt) S.key[i] = 2u * nbv[j] + (nbv[j] != b0 + base + loc[j] ? 1u : 0u);
        }
    } else {
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const int i = tid * IPT + j;
            if (i < cnt) S.key[i] = 2u * nbv[j] + 1u;
        }
    }
    __syncthreads();

    // key range of the tile -> number of radix passes
    uint32_t kmin = 0xffffffffu, kmax = 0;
    for (int i = tid; i < cnt; i += RB_THREADS) {
        kmin = min(kmin, S.key[i]);
        kmax = max(kmax, S.key[i]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, o, 64));
        kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, o, 64));
    }
    if (tid == 0) { S.misc[2] = 0xffffffffu; S.misc[3] = 0; }
    __syncthreads();
    if ((tid & 63) == 0) {
        atomicMin(&S.misc[2], kmin);
        atomicMax(&S.misc[3], kmax);
    }
    __syncthreads();
    kmin = S.misc[2];
    kmax = S.misc[3];
    const uint32_t span = kmax - kmin;
    const int bits = span ? 32 - __clz(span) : 0;
    const int passes = (bits + RADIX - 1) / RADIX;

    for (int i = tid; i < TILE; i += RB_THREADS) {
        if (i < cnt) S.key[i] -= kmin;
        S.item[0][i] = (uint16_t)i;
    }
    __syncthreads();

    // LSD radix passes: thread t owns the contiguous slots [t*IPT, (t+1)*IPT)
    // of the current order, so ranks within a digit follow slot order.
    int cur = 0;
    for (int ps = 0; ps < passes; ++ps) {
        const int shift = ps * RADIX;
        constexpr int NW = DIG / 8;                       // 64-bit words of 8-bit counters
        uint8_t dig[IPT], rk[IPT];
        uint16_t it[IPT];
#pragma unroll
        for (int j = 0; j < IPT; ++j) it[j] = S.item[cur][tid * IPT + j];
#pragma unroll
        for (int j = 0; j < IPT; ++j)                      // padding slots sort last
            dig[j] = (uint8_t)(tid * IPT + j < cnt ? (S.key[it[j]] >> shift) & (DIG - 1) : DIG - 1);
        uint64_t cw[NW];
#pragma unroll
        for (int q = 0; q < NW; ++q) cw[q] = 0;
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const int w = dig[j] >> 3, sh = (dig[j] & 7) * 8;
            uint64_t word = cw[0];
#pragma unroll
            for (int q = 1; q < NW; ++q) word = w == q ? cw[q] : word;
            rk[j] = (uint8_t)((word >> sh) & 0xffu);
#pragma unroll
            for (int q = 0; q < NW; ++q)
                if (w == q) cw[q] += 1ull << sh;
        }
#pragma unroll
        for (int dg = 0; dg < DIG; ++dg)
            S.cnt[cpad(dg * RB_THREADS + tid)] = (uint32_t)((cw[dg >> 3] >> ((dg & 7) * 8)) & 0xffu);
        __syncthreads();
        // exclusive scan over (digit, thread) in digit-major order: thread t
        // owns the flattened counters [t*DIG, (t+1)*DIG)
        uint32_t v[DIG];
        uint32_t sum = 0;
#pragma unroll
        for (int j = 0; j < DIG; ++j) {
            v[j] = S.cnt[cpad(tid * DIG + j)];
            sum += v[j];
        }
        uint32_t tot;
        uint32_t base = block_excl_scan(sum, S.wsum, &tot);
#pragma unroll
        for (int j = 0; j < DIG; ++j) {
            S.cnt[cpad(tid * DIG + j)] = base;
            base += v[j];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const uint32_t pos = S.cnt[cpad(dig[j] * RB_THREADS + tid)] + rk[j];
            S.item[cur ^ 1][pos] = it[j];
        }
        __syncthreads();
        cur ^= 1;
    }

    // runs of equal key in sorted order
    uint32_t head[IPT];
    uint32_t nh = 0;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int slot = tid * IPT + j;
        uint32_t h = 0;
        if (slot < cnt) {
            const uint32_t k = S.key[S.item[cur][slot]];
            h = (slot == 0) || (k != S.key[S.item[cur][slot - 1]]);
        }
        head[j] = h;
        nh += h;
    }
    uint32_t n_runs;
    uint32_t rbase = block_excl_scan(nh, S.wsum, &n_runs);
    // run start positions into S.cnt, then counts
    uint32_t r = rbase;
#pragma unroll
    for (int j = 0; j < IPT; ++j)
        if (head[j]) S.cnt[r++] = (uint32_t)(tid * IPT + j);
    if (tid == 0) S.cnt[n_runs] = (uint32_t)cnt;
    __syncthreads();
    const int64_t rt = tile * TILE;
    for (uint32_t q = tid; q < n_runs; q += RB_THREADS) {
        const uint32_t st = S.cnt[q], len = S.cnt[q + 1] - st;
        const uint32_t key = S.key[S.item[cur][st]] + kmin;
        sc.run_key[rt + q] = key;
        sc.run_info[rt + q] = st | (len << 16);
        atomicAdd(&sc.key_cnt[key], len);
        atomicAdd(&sc.key_nruns[key], 1u);
    }
    if (tid == 0) sc.tile_nruns[tile] = n_runs;
    n_runs_out = n_runs;
    return cur;
}

template <int IPT, int RADIX>
__global__ __launch_bounds__(RB_THREADS) void k_rebin_tiles(const uint32_t *new_bin, const int64_t *old_start,
                                                           int64_t n, uint32_t n_bins, RebinScratch sc,
                                                           uint32_t *status) {
    constexpr int TILE = RB_THREADS * IPT;
    __shared__ TileSmem<IPT, RADIX, false> S;
    const int tid = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const int64_t lo = tile * TILE;
    const int cnt = (int)min((int64_t)TILE, n - lo);
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int i = tid + j * RB_THREADS;
        if (i < cnt) S.key[i] = new_bin[lo + i];
    }
    __syncthreads();
    uint32_t n_runs;
    const int cur = tile_sort_emit<IPT, RADIX, false>(S, old_start, tile, cnt, n_bins, sc, status, n_runs);
    for (int i = tid; i < cnt; i += RB_THREADS) sc.perm[lo + i] = S.item[cur][i];
}

// Pass 2: single-pass scan (decoupled look-back) of the per-key (count, runs)
// pairs.  Each 64-bit state word holds flag << 62 | count << 31 | runs; the
// state words are relaxed atomics, since a block reads nothing of its
// predecessors but those words.

__global__ __launch_bounds__(256) void k_rebin_scan(uint32_t n_keys, uint32_t n_bins, int64_t n, RebinScratch sc,
                                                    int64_t *new_start, uint32_t *status) {
    __shared__ uint32_t s_wsum[4];
    __shared__ uint64_t s_excl;
    __shared__ uint32_t s_bid;
    const int tid = threadIdx.x;
    if (tid == 0) s_bid = atomicAdd(sc.scan_ctr, 1u);
    __syncthreads();
    const uint32_t bid = s_bid;
    const uint64_t k0 = (uint64_t)bid * SCAN_TILE + (uint64_t)tid * SCAN_IPT;
    uint32_t c[SCAN_IPT], r[SCAN_IPT];
    uint32_t cs = 0, rsum = 0;
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) {
        const uint64_t k = k0 + j;
        c[j] = r[j] = 0;
        if (k < n_keys) {
            c[j] = sc.key_cnt[k];
            r[j] = sc.key_nruns[k];
        }
        cs += c[j];
        rsum += r[j];
    }
    uint32_t ctot, rtot;
    uint32_t cex = block_excl_scan(cs, s_wsum, &ctot);
    uint32_t rex = block_excl_scan(rsum, s_wsum, &rtot);
    if (tid == 0) {
        const uint64_t agg = ((uint64_t)ctot << 31) | rtot;
        uint64_t excl = 0;
        if (bid == 0) {
            __hip_atomic_store(&sc.scan_state[0], ST_PRE | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(&sc.scan_state[bid], ST_AGG | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int64_t j = (int64_t)bid - 1;
            uint32_t spins = 0;
            while (j >= 0) {
                const uint64_t st = __hip_atomic_load(&sc.scan_state[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((st >> 62) == 0) {
                    if (++spins > (1u << 26)) {   // bounded wait: report instead of hanging
                        atomicOr(status, PIC_DEV_RANGE);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                const uint64_t v = st & ST_VAL;
                excl = ((((excl >> 31) + (v >> 31)) & 0x7fffffffull) << 31) |
                       (((excl & 0x7fffffffull) + (v & 0x7fffffffull)) & 0x7fffffffull);
                if ((st >> 62) == 2) break;
                --j;
            }
            const uint64_t incl = ((((excl >> 31) + ctot) & 0x7fffffffull) << 31) |
                                  (((excl & 0x7fffffffull) + rtot) & 0x7fffffffull);
            __hip_atomic_store(&sc.scan_state[bid], ST_PRE | incl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        s_excl = excl;
    }
    __syncthreads();
    uint32_t cb = (uint32_t)(s_excl >> 31) + cex, rb = (uint32_t)(s_excl & 0x7fffffffull) + rex;
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) {
        const uint64_t k = k0 + j;
        if (k < n_keys) {
            sc.key_base[k] = cb;
            sc.list_off[k] = rb;
            if ((k & 1) == 0) new_start[k >> 1] = cb;
        }
        cb += c[j];
        rb += r[j];
        if (k + 1 == n_keys) {
            sc.list_off[n_keys] = rb;
            new_start[n_bins] = n;
        }
    }
}

// Pass 3a: append every run to the list of its key (slot order arbitrary).
__global__ __launch_bounds__(256) void k_rebin_lists(RebinScratch sc, int tile_slots) {
    const int64_t tile = blockIdx.x;
    const uint32_t nr = sc.tile_nruns[tile];
    for (uint32_t q = threadIdx.x; q < nr; q += blockDim.x) {
        const uint32_t a = (uint32_t)(tile * tile_slots + q);
        const uint32_t key = sc.run_key[a];
        const uint32_t slot = sc.list_off[key] + atomicAdd(&sc.key_fill[key], 1u);
        sc.list[slot] = a;
    }
}

__global__ __launch_bounds__(256) void k_rebin_place(RebinScratch sc, uint32_t n_keys) {
    const int lane = threadIdx.x & 63;
    const int grp = lane >> 4, sub = lane & 15;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t k0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 4; k0 < n_keys;
         k0 += waves * 4) {
        const int64_t key = k0 + grp;
        uint32_t l0 = 0, len = 0, kb = 0;
        if (key < n_keys) {
            l0 = sc.list_off[key];
            len = sc.list_off[key + 1] - l0;
            kb = sc.key_base[key];
        }
        if (len <= 16) place_sorted<16>(sc, sc.list, l0, len, kb, sub);   // len 0: nothing written
        // keys with longer lists: whole wavefront, one after the other
        for (int g = 0; g < 4; ++g) {
            const uint32_t gl0 = (uint32_t)__shfl((int)l0, g * 16, 64);
            const uint32_t glen = (uint32_t)__shfl((int)len, g * 16, 64);
            const uint32_t gkb = (uint32_t)__shfl((int)kb, g * 16, 64);
            if (glen <= 16) continue;
            if (glen <= 64) {
                place_sorted<64>(sc, sc.list, gl0, glen, gkb, lane);
            } else {
                for (uint32_t q = lane; q < glen; q += 64) {
                    const uint32_t a = sc.list[gl0 + q];
                    uint32_t before = 0;
                    for (uint32_t j = gl0; j < gl0 + glen; ++j) {
                        const uint32_t bb = sc.list[j];
                        if (bb < a) before += sc.run_info[bb] >> 16;
                    }
                    sc.run_dest[a] = gkb + before;
                }
            }
        }
    }
}

// Pass 4: scatter.  Mode 0 stages each column of the tile through LDS:
// thread t loads the slots t + 256 i in old order (coalesced), and after a
// barrier writes the sorted slots t + 256 i, so a wavefront writes 64
// consecutive sorted slots, i.e. consecutive destinations inside a run.  All
// global loads of the tile (run table, permutation, up to four columns) are
// issued before the first one is waited for, so a block pays one memory
// latency instead of one per step.  Mode 1 does not stage: each sorted slot
// loads its record straight from the tile (an L2-resident window).
template <typename T, bool NT>
__device__ __forceinline__ void put_out(T *p, T v) {
    if (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

template <int IPT, int MODE, bool NT, int SC_GROUP>
__global__ __launch_bounds__(RB_THREADS) void k_rebin_scatter(int64_t n, RebinScratch sc, Cols cols,
                                                             uint32_t *status) {
    constexpr int TILE = RB_THREADS * IPT;
    __shared__ uint16_t s_rstart[TILE + 1];
    __shared__ uint32_t s_rdest[TILE];
    __shared__ uint64_t s_stage[MODE == 0 ? TILE : 1];
    const int tid = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const int64_t lo = tile * TILE;
    const int cnt = (int)min((int64_t)TILE, n - lo);
    // speculative run-table loads (the first 256 entries of the tile's area
    // are always in range), issued together with the rest
    const uint32_t nr = sc.tile_nruns[tile];
    const uint32_t ri0 = sc.run_info[lo + tid];
    const uint32_t rd0 = sc.run_dest[lo + tid];
    uint16_t src[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int j = tid + i * RB_THREADS;
        src[i] = j < cnt ? sc.perm[lo + j] : (uint16_t)0;
    }
    uint64_t val[SC_GROUP][IPT];
    const int ng = min(cols.n, SC_GROUP);
    if (MODE == 0) {
#pragma unroll
        for (int c = 0; c < SC_GROUP; ++c) {
            if (c >= ng) break;
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                const int j = tid + i * RB_THREADS;
                val[c][i] = 0;
                if (j < cnt)
                    val[c][i] = cols.bytes[c] == 8 ? ((const uint64_t *)cols.in[c])[lo + j]
                                                   : (uint64_t)((const uint32_t *)cols.in[c])[lo + j];
            }
        }
    }
    if ((uint32_t)tid < nr) {
        s_rstart[tid] = (uint16_t)(ri0 & 0xffffu);
        s_rdest[tid] = rd0;
    }
    for (uint32_t q = tid + RB_THREADS; q < nr; q += RB_THREADS) {
        s_rstart[q] = (uint16_t)(sc.run_info[lo + q] & 0xffffu);
        s_rdest[q] = sc.run_dest[lo + q];
    }
    if (tid == 0) s_rstart[nr] = (uint16_t)min(cnt, 0xffff);
    __syncthreads();
    uint32_t dst[IPT];
#pragma unroll
    for (int i = 0; i < IPT; ++i) {
        const int j = tid + i * RB_THREADS;
        dst[i] = 0xffffffffu;
        if (j < cnt) {
            // run holding sorted slot j: last run start <= j
            uint32_t a = 0, b = nr - 1;
            while (a < b) {
                const uint32_t m = (a + b + 1) >> 1;
                if (s_rstart[m] <= j) a = m; else b = m - 1;
            }
            dst[i] = s_rdest[a] + (uint32_t)(j - s_rstart[a]);
            if (dst[i] >= (uint32_t)n) {        // inconsistent input: drop, never write out of range
                dst[i] = 0xffffffffu;
                flag_status(status, PIC_DEV_RANGE);
            }
        }
    }
    if (MODE == 1) {
        for (int c = 0; c < cols.n; ++c) {
            if (cols.bytes[c] == 8) {
                const uint64_t *in = (const uint64_t *)cols.in[c] + lo;
                uint64_t *out = (uint64_t *)cols.out[c];
                uint64_t v[IPT];
#pragma unroll
                for (int i = 0; i < IPT; ++i) v[i] = dst[i] != 0xffffffffu ? in[src[i]] : 0;
#pragma unroll
                for (int i = 0; i < IPT; ++i)
                    if (dst[i] != 0xffffffffu) put_out<uint64_t, NT>(&out[dst[i]], v[i]);
            } else {
                const uint32_t *in = (const uint32_t *)cols.in[c] + lo;
                uint32_t *out = (uint32_t *)cols.out[c];
                uint32_t v[IPT];
#pragma unroll
                for (int i = 0; i < IPT; ++i) v[i] = dst[i] != 0xffffffffu ? in[src[i]] : 0;
#pragma unroll
                for (int i = 0; i < IPT; ++i)
                    if (dst[i] != 0xffffffffu) put_out<uint32_t, NT>(&out[dst[i]], v[i]);
            }
        }
        return;
    }
    for (int c0 = 0; c0 < cols.n; c0 += SC_GROUP) {
        if (c0 > 0) {                                   // further groups: load them now
#pragma unroll
            for (int c = 0; c < SC_GROUP; ++c) {
                if (c0 + c >= cols.n) break;
#pragma unroll
                for (int i = 0; i < IPT; ++i) {
                    const int j = tid + i * RB_THREADS;
                    val[c][i] = 0;
                    if (j < cnt)
                        val[c][i] = cols.bytes[c0 + c] == 8 ? ((const uint64_t *)cols.in[c0 + c])[lo + j]
                                                            : (uint64_t)((const uint32_t *)cols.in[c0 + c])[lo + j];
                }
            }
        }
#pragma unroll
        for (int c = 0; c < SC_GROUP; ++c) {
            if (c0 + c >= cols.n) break;
#pragma unroll
            for (int i = 0; i < IPT; ++i) s_stage[tid + i * RB_THREADS] = val[c][i];
            __syncthreads();
            if (cols.bytes[c0 + c] == 8) {
                uint64_t *out = (uint64_t *)cols.out[c0 + c];
#pragma unroll
                for (int i = 0; i < IPT; ++i)
                    if (dst[i] != 0xffffffffu) put_out<uint64_t, NT>(&out[dst[i]], s_stage[src[i]]);
            } else {
                uint32_t *out = (uint32_t *)cols.out[c0 + c];
#pragma unroll
                for (int i = 0; i < IPT; ++i)
                    if (dst[i] != 0xffffffffu) put_out<uint32_t, NT>(&out[dst[i]], (uint32_t)s_stage[src[i]]);
            }
            __syncthreads();
        }
    }
}

// Zero the per-call counters and, when the input is sorted, find the old bins
// covering each tile (one kernel instead of two).
__global__ void k_rebin_prep(uint32_t *zero, int64_t n_zero, const int64_t *old_start, int64_t n_bins, int64_t n,
                             int tile, RebinScratch sc) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = gid; i < n_zero; i += stride) zero[i] = 0;
    if (!old_start) return;
    const int64_t n_tiles = (n + tile - 1) / tile;
    for (int64_t b = gid; b < n_bins; b += stride) {
        const int64_t s0 = max(old_start[b], (int64_t)0), s1 = min(old_start[b + 1], n);
        if (s1 <= s0) continue;
        for (int64_t t = (s0 + tile - 1) / tile; t * tile < s1; ++t) sc.tile_bin[2 * t] = (uint32_t)b;
        for (int64_t t = s0 / tile; t < n_tiles; ++t) {
            const int64_t last = min((t + 1) * tile, n) - 1;
            if (last >= s1) break;
            if (last >= s0) sc.tile_bin[2 * t + 1] = (uint32_t)(b + 1);
        }
        // the bin of every 64th slot (a wavefront's first slot)
        for (int64_t c = (s0 + 63) >> 6; (c << 6) < s1; ++c) sc.wave_bin[c] = (uint32_t)b;
    }
}

// ----------------------------------------------------------------- launchers

size_t rebin_scratch_bytes(const pic_tree *t, int64_t n, int scheme) {
    // large enough for every supported tile size
    const int64_t nb = n_bins_of(t, scheme);
    // the 2D fused step deposits in its writing pass: one partial per run
    const int ns = t->dim == 2 ? (scheme == PIC_PIT ? 4 : 9) : 0;
    return std::max({rebin_layout(n, nb, 1024, ns).total, rebin_layout(n, nb, 2048, ns).total,
                     rebin_layout(n, nb, 4096).total});
}

template <int IPT>
static void launch_tiles(int radix, dim3 g, hipStream_t s, const uint32_t *nb, const int64_t *os, int64_t n,
                         uint32_t n_bins, const RebinScratch &sc, uint32_t *status) {
    if (radix == 5) PIC_LAUNCH("rebin_tiles", (k_rebin_tiles<IPT, 5>), g, dim3(RB_THREADS), 0, s, nb, os, n, n_bins, sc, status);
    else PIC_LAUNCH("rebin_tiles", (k_rebin_tiles<IPT, 4>), g, dim3(RB_THREADS), 0, s, nb, os, n, n_bins, sc, status);
}

template <int IPT, int MODE, bool NT>
static void launch_scatter_g(const Tuning &tu, dim3 g, hipStream_t s, int64_t n, const RebinScratch &sc,
                             const Cols &cols, uint32_t *status) {
    switch (tu.scatter_group) {
        case 1: PIC_LAUNCH("rebin_scatter", (k_rebin_scatter<IPT, MODE, NT, 1>), g, dim3(RB_THREADS), 0, s, n, sc, cols, status); break;
        case 2: PIC_LAUNCH("rebin_scatter", (k_rebin_scatter<IPT, MODE, NT, 2>), g, dim3(RB_THREADS), 0, s, n, sc, cols, status); break;
        default: PIC_LAUNCH("rebin_scatter", (k_rebin_scatter<IPT, MODE, NT, 4>), g, dim3(RB_THREADS), 0, s, n, sc, cols, status); break;
    }
}

template <int IPT>
static void launch_scatter(const Tuning &tu, int mode, dim3 g, hipStream_t s, int64_t n, const RebinScratch &sc,
                           const Cols &cols, uint32_t *status) {
    const bool nt = tu.scatter_nt != 0;
    if (mode == 1) {
        if (nt) launch_scatter_g<IPT, 1, true>(tu, g, s, n, sc, cols, status);
        else launch_scatter_g<IPT, 1, false>(tu, g, s, n, sc, cols, status);
    } else {
        if (nt) launch_scatter_g<IPT, 0, true>(tu, g, s, n, sc, cols, status);
        else launch_scatter_g<IPT, 0, false>(tu, g, s, n, sc, cols, status);
    }
}

// The part of a re-bin that follows the tile sort: per-key scan, run lists,
// run placement.
static void launch_rebin_middle(const pic_tree *t, int64_t n, int64_t n_bins, int tile, const RebinScratch &sc,
                                int64_t *new_start, hipStream_t s) {
    const int64_t keys = 2 * n_bins;
    const int64_t tiles = (n + tile - 1) / tile;
    const int64_t scan_blocks = (keys + SCAN_TILE - 1) / SCAN_TILE;
    PIC_LAUNCH("rebin_scan", k_rebin_scan, dim3(scan_blocks), dim3(256), 0, s, (uint32_t)keys, (uint32_t)n_bins, n, sc,
               new_start, t->dt.status);
    if (n > 0) {
        PIC_LAUNCH("rebin_lists", k_rebin_lists, dim3(tiles), dim3(256), 0, s, sc, tile);
        PIC_LAUNCH("rebin_place", k_rebin_place, dim3(grid_for(keys, 16, 1 << 16)), dim3(256), 0, s, sc, (uint32_t)keys);
    }
}

hipError_t launch_rebin(const pic_tree *t, int scheme, int64_t n, const uint32_t *new_bin, const int64_t *old_start,
                        const Cols &cols, int64_t *new_start, void *scratch, size_t scratch_bytes, hipStream_t s) {
    const int64_t n_bins = n_bins_of(t, scheme);
    const int ipt = t->tune.rebin_ipt;
    const int tile = RB_THREADS * ipt;
    const RebinLayout L = rebin_layout(n, n_bins, tile);
    if (scratch_bytes < L.total) return hipErrorInvalidValue;
    char *base = (char *)scratch;
    const RebinScratch sc = bind_scratch(L, base);
    const int64_t tiles = (n + tile - 1) / tile;
    // counters, scan flags and the block counter start at zero (a kernel, not a
    // memset node, so the sequence can be captured in a graph); the same kernel
    // finds the old bins covering each tile
    const int64_t zero_words = (int64_t)((L.key_base - L.key_cnt) / 4);
    PIC_LAUNCH("rebin_prep", k_rebin_prep, dim3(grid_for(std::max(zero_words, n_bins), 256, 4096)), dim3(256), 0,
               s, (uint32_t *)(base + L.key_cnt), zero_words, n > 0 ? old_start : nullptr, n_bins, n, tile, sc);
    if (n > 0) {
        if (ipt == 8) launch_tiles<8>(t->tune.rebin_radix, dim3(tiles), s, new_bin, old_start, n, (uint32_t)n_bins, sc, t->dt.status);
        else launch_tiles<16>(t->tune.rebin_radix, dim3(tiles), s, new_bin, old_start, n, (uint32_t)n_bins, sc, t->dt.status);
    }
    launch_rebin_middle(t, n, n_bins, tile, sc, new_start, s);
    if (n > 0) {
        if (ipt == 8) launch_scatter<8>(t->tune, t->tune.scatter_mode, dim3(tiles), s, n, sc, cols, t->dt.status);
        else launch_scatter<16>(t->tune, t->tune.scatter_mode, dim3(tiles), s, n, sc, cols, t->dt.status);
    }
    return hipGetLastError();
}

void launch_prep(uint32_t *zero, int64_t n_zero, const int64_t *old_start, int64_t n_bins, int64_t n, int tile,
                 const RebinScratch &sc, hipStream_t s) {
    PIC_LAUNCH("rebin_prep", k_rebin_prep, dim3(grid_for(std::max(n_zero, old_start ? n_bins : 0), 256, 4096)),
               dim3(256), 0, s, zero, n_zero, old_start, n_bins, n, tile, sc);
}

}  // namespace pic
