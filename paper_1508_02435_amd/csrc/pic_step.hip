// pic_step.hip -- the fused FP64 step (pic_step): a key pass pushes every
// particle and writes its key 2*bin + arrived; the ranking, scan and
// placement passes (pic_rank.hip) give every (tile, key) run its
// destination; an emit pass pushes every particle again (the same
// arithmetic, so the same state and bin) and writes it to its run's
// destination plus its rank, in tile-sorted order through LDS; then the
// deposit on the re-binned set.
#include <hip/hip_runtime.h>

#include "pic_launch.h"

namespace pic {

// Key pass of the unfused form: one particle per thread, pushed, its key
// 2*bin + arrived written out; with `store` the pushed state also goes back
// to the input arrays, in place, so that the writing pass only moves it.
// It also clears the per-call counters.  Its loads wait on one another
// (old bin, field, rank tables), so it wants resident wavefronts: at least
// five per SIMD, which holds the 3D forms to 72 registers (seven resident).
template <int D, int SCHEME, bool REG, bool MULTI, int MOVE>
__global__ __launch_bounds__(256, 5) void k_step_key(DevTree t, DevInst in0, F64Ptrs P, int64_t n, double qmdt0,
                                                  double dt0, const double *qa, const double *da,
                                                  const int64_t *inst_start, const int64_t *old_start,
                                                  uint32_t n_bins, uint32_t *key_out, uint32_t *zero,
                                                  int64_t n_zero, int store, int flops) {
    __shared__ int32_t lds[REG ? 1 : PIC_LDS_NODES];
    const int lds_n = MULTI ? 0 : stage_nodes<REG>(t, in0, lds);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_zero; i += stride) zero[i] = 0u;
    // one block per 256 particles when the grid covers the set: the blocks
    // of the leapfrog push walk the writing pass's XCD chunks backwards
    // (xcd_tile_rev).  Not for adaptive 2D trees, whose key pass (a descent
    // per particle) runs faster forwards (0.181 instead of 0.196 ms on the
    // adaptive 2D workload), nor for free streaming, which runs faster
    // forwards too (0.108 instead of 0.117 ms in 3D; with 4096 artificial
    // flops per move, before that chain was unrolled, 1.23 instead of 2.15).
    const bool one_pass = MOVE == MOVE_PUSH && (D == 3 || REG) && stride >= n;
    const int64_t b0 = one_pass ? xcd_tile_rev(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    for (int64_t p = b0 * blockDim.x + threadIdx.x; p < n; p += one_pass ? n : stride) {
        uint32_t bad = 0;
        double xv[D], vv[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            xv[k] = P.x[k][p];
            vv[k] = P.v[k][p];
        }
        key_out[p] = step_key_one<D, SCHEME, REG, MULTI, MOVE>(t, in0, P, p, xv, vv, qmdt0, dt0, qa, da,
                                                               inst_start, old_start, n_bins, lds, lds_n, bad, flops);
        if (store) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                P.x[k][p] = xv[k];
                P.v[k][p] = vv[k];
            }
        }
        if (bad) flag_status(t.status, bad);
    }
}

// ------------------------------------------------- deposit in the writing pass

__device__ __forceinline__ double readlane_f64(double x, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    return __hiloint2double(hi, lo);
}

// Tile-local sorted start and sorted-list position of run rid of the tile at
// lo.  Read at run ends only (a few per wavefront), from the run tables.
__device__ __forceinline__ uint32_t run_start_of(const uint32_t *run_info, int64_t lo, uint32_t rid) {
    return run_info[lo + rid] & 0xffffu;
}
__device__ __forceinline__ uint32_t run_place_of(const uint32_t *run_pos, int64_t lo, uint32_t rid) {
    return run_pos[lo + rid];
}

constexpr uint32_t EDGE_NONE = 0xffffu, EDGE_VALID = 1u << 16, EDGE_CONT = 1u << 17;

// A run ending in wavefront w (first sorted slot wq0): its sum is complete
// when the run started in w; otherwise it is w's first piece of the run.
template <int NSD>
__device__ __forceinline__ void emit_finish(uint32_t r, const double (&v)[NSD], uint32_t wq0, int w,
                                            double (*s_edge)[2][NSD], uint32_t (*s_erid)[2], int64_t lo,
                                            const uint32_t *run_info, const uint32_t *run_pos, double *run_part) {
    if (run_start_of(run_info, lo, r) >= wq0) {
        double *o = run_part + (int64_t)run_place_of(run_pos, lo, r) * NSD;
#pragma unroll
        for (int c = 0; c < NSD; ++c) o[c] = v[c];
    } else {
#pragma unroll
        for (int c = 0; c < NSD; ++c) s_edge[w][0][c] = v[c];
        s_erid[w][0] = r | EDGE_VALID;
    }
}

// One wavefront's share of the writing pass's deposit: its sorted slots
// [64 IPT w, 64 IPT (w+1)) in rounds of 64 (positions staged in s_val[0..D)).
// One step of a segmented inclusive scan over a wavefront: each lane of the
// rows in ROWS takes the partial sums of the lane that the DPP pattern CTRL
// names when both carry the same run id.  Runs are contiguous, so equal ids
// at both ends of a step mean one run; a lane with no source (shifted in
// from outside its row, or a row left out) sees an id no run has.
template <int CTRL, int ROWS, int NSD>
__device__ __forceinline__ void seg_step(uint32_t rid, double (&acc)[NSD]) {
    const uint32_t orid = (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)rid, CTRL, ROWS, 0xf, false);
    const bool take = orid == rid;
#pragma unroll
    for (int c = 0; c < NSD; ++c) {
        const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(acc[c]), CTRL, ROWS, 0xf, false);
        const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(acc[c]), CTRL, ROWS, 0xf, false);
        if (take) acc[c] = __dadd_rn(__hiloint2double(hi, lo), acc[c]);
    }
}

template <int D, int SCHEME, int TILE, int NT, int NSD>
__device__ __forceinline__ void emit_deposit(const DevInst &in, const uint64_t (*s_val)[TILE], const uint16_t *s_rid,
                                             double (*s_edge)[2][NSD], uint32_t (*s_erid)[2], int64_t lo, int cnt,
                                             const uint32_t *run_info, const uint32_t *run_pos, double *run_part) {
    constexpr int IPT = TILE / NT;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t wq0 = (uint32_t)w * 64u * IPT, wq1 = wq0 + 64u * IPT;
    double carry[NSD];
#pragma unroll
    for (int c = 0; c < NSD; ++c) carry[c] = 0.0;
    uint32_t crid = EDGE_NONE;
#pragma unroll
    for (int r = 0; r < IPT; ++r) {
        const uint32_t qq = wq0 + 64u * r + lane;
        const bool valid = qq < (uint32_t)cnt;
        const uint32_t rid = valid ? (uint32_t)s_rid[qq] : EDGE_NONE;
        double acc[NSD];
#pragma unroll
        for (int c = 0; c < NSD; ++c) acc[c] = 0.0;
        if (valid) {
            double xp[D];
#pragma unroll
            for (int k = 0; k < D; ++k) xp[k] = __longlong_as_double((long long)s_val[k][qq]);
            deposit_one<D, SCHEME, true, NSD>(in, xp, 0, 1.0, 1u, 1.0, 1.0, false, acc);
        }
        // the previous round's last run: continued by this round, or ended there
        if (crid != EDGE_NONE) {
            const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)rid, 0);
            if (r0 == crid) {
                if (lane == 0)
#pragma unroll
                    for (int c = 0; c < NSD; ++c) acc[c] = __dadd_rn(carry[c], acc[c]);
            } else if (lane == 0) {
                emit_finish<NSD>(crid, carry, wq0, w, s_edge, s_erid, lo, run_info, run_pos, run_part);
            }
        }
        // segmented inclusive scan across the lanes: shifts by 1, 2, 4, 8
        // inside rows of 16 lanes, then each row's last lane to the next row
        // and lane 31 to the upper half (DPP moves: no LDS traffic)
        seg_step<0x111, 0xf>(rid, acc);   // row_shr:1
        seg_step<0x112, 0xf>(rid, acc);   // row_shr:2
        seg_step<0x114, 0xf>(rid, acc);   // row_shr:4
        seg_step<0x118, 0xf>(rid, acc);   // row_shr:8
        seg_step<0x142, 0xa>(rid, acc);   // row_bcast:15 into rows 1 and 3
        seg_step<0x143, 0xc>(rid, acc);   // row_bcast:31 into rows 2 and 3
        const uint32_t nrid = (uint32_t)__shfl_down((int)rid, 1, 64);
        if (valid && lane < 63 && nrid != rid)
            emit_finish<NSD>(rid, acc, wq0, w, s_edge, s_erid, lo, run_info, run_pos, run_part);
        crid = (uint32_t)__builtin_amdgcn_readlane((int)rid, 63);
#pragma unroll
        for (int c = 0; c < NSD; ++c) carry[c] = readlane_f64(acc[c], 63);
    }
    if (crid != EDGE_NONE && lane == 0) {   // the wavefront's last run
        const bool cont = wq1 < (uint32_t)cnt && (uint32_t)s_rid[wq1] == crid;
        if (!cont) {
            emit_finish<NSD>(crid, carry, wq0, w, s_edge, s_erid, lo, run_info, run_pos, run_part);
        } else if (run_start_of(run_info, lo, crid) >= wq0) {
#pragma unroll
            for (int c = 0; c < NSD; ++c) s_edge[w][1][c] = carry[c];
            s_erid[w][1] = crid | EDGE_VALID;
        } else {
#pragma unroll
            for (int c = 0; c < NSD; ++c) s_edge[w][0][c] = carry[c];
            s_erid[w][0] = crid | EDGE_VALID | EDGE_CONT;
        }
    }
}

// Runs crossing wavefronts: the wavefront a run started in (thread w) adds
// the pieces of the following wavefronts in order.
template <int NW, int NSD>
__device__ __forceinline__ void emit_edges(const double (*s_edge)[2][NSD], const uint32_t (*s_erid)[2], int64_t lo,
                                           const uint32_t *run_pos, double *run_part, uint32_t *status) {
    const int w = threadIdx.x;
    const uint32_t e = s_erid[w][1];
    if (!(e & EDGE_VALID)) return;
    const uint32_t r = e & 0xffffu;
    double sum[NSD];
#pragma unroll
    for (int c = 0; c < NSD; ++c) sum[c] = s_edge[w][1][c];
    for (int w2 = w + 1; w2 < NW; ++w2) {
        const uint32_t f = s_erid[w2][0];
        if (!(f & EDGE_VALID) || (f & 0xffffu) != r) {   // cannot happen for a consistent run table
            atomicOr(status, PIC_DEV_RANGE);
            break;
        }
#pragma unroll
        for (int c = 0; c < NSD; ++c) sum[c] = __dadd_rn(sum[c], s_edge[w2][0][c]);
        if (!(f & EDGE_CONT)) break;
    }
    double *o = run_part + (int64_t)run_place_of(run_pos, lo, r) * NSD;
#pragma unroll
    for (int c = 0; c < NSD; ++c) o[c] = sum[c];
}

// Emit pass: slot p of tile T writes its pushed state to
// run_dest[T's run area + rid] + rank.  NT threads cover the TILE slots of a
// tile.  The tile's records are first put in tile-local sorted order (runs
// one after the other, each run at its start from the run table) through
// LDS, two columns at a time, so that a wavefront's stores cover
// consecutive destinations of a few runs instead of a few elements of each of
// many runs.
//
// With DEP (2D, regular single trees, uniform charge) the pass deposits as
// well (paper Sec. 3 step 1).  Once the positions are in LDS in sorted order,
// wavefront w takes the sorted slots [64 IPT w, 64 IPT (w+1)) in rounds of
// 64, computes each slot's corner (PIT) or stencil (PIDT) weights and sums
// them per run with a segmented inclusive scan across the lanes (a fixed
// tree of lane shuffles; runs are contiguous in sorted order, so equal run
// ids at both ends of a step mean one segment), the last lane's run carried
// into the next round.  A run that ends inside the wavefront and started in
// it is complete: its sum goes to run_part at the run's position among all
// runs sorted by (key, tile).  A run crossing wavefronts leaves one piece per
// wavefront; the wavefront it started in adds the later pieces in wavefront
// order.  No float atomics: every sum has a fixed order.  k_deposit_runs
// then adds each bin's runs in output order.
template <int D, int SCHEME, bool REG, bool MULTI, int TILE, int NT, bool DEP, int MOVE>
__global__ __launch_bounds__(NT) void k_step_emit(DevTree t, DevInst in0, F64Ptrs P, int64_t n, double qmdt0,
                                                  double dt0, const double *qa, const double *da,
                                                  const int64_t *inst_start, const uint32_t *meta,
                                                  const uint32_t *run_dest, const uint32_t *run_info,
                                                  const uint32_t *run_pos, double *run_part, F64Ptrs out,
                                                  Cols extra, int xcd) {
    constexpr bool PUSHED = MOVE == MOVE_STORED;   // the key pass stored the moved state
    constexpr int IPT = TILE / NT;
    constexpr int NW = NT / 64;
    constexpr int NSD = SCHEME == PIC_PIT ? (1 << D) : (D == 2 ? 9 : 27);
    static_assert(!DEP || (D == 2 && REG && !MULTI), "the writing pass deposits for 2D regular single trees");
    __shared__ int32_t lds[REG ? 1 : PIC_LDS_NODES];
    // columns staged per barrier pair: two, one for 4096-particle tiles (LDS)
    constexpr int SC = TILE > 2048 ? 1 : 2;
    static_assert(!DEP || SC == 2, "the writing-pass deposit needs both position columns staged at once");
    __shared__ uint64_t s_val[SC][TILE];
    __shared__ uint32_t s_dst[TILE];
    __shared__ uint32_t s_rd[RUN_HEAD], s_ro[RUN_HEAD];
    __shared__ uint16_t s_rid[DEP ? TILE : 1];
    __shared__ double s_edge[DEP ? NW : 1][2][DEP ? NSD : 1];   // per wavefront: first piece, last piece
    __shared__ uint32_t s_erid[DEP ? NW : 1][2];                // their run ids | VALID | CONT
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t lo = xcd_tile(blockIdx.x, gridDim.x, xcd) * TILE;
    const int lds_n = (MULTI || PUSHED) ? 0 : stage_nodes<REG>(t, in0, lds);
    const int64_t base = lo + (int64_t)w * 64 * IPT + lane;
    const int cnt = (int)min((int64_t)TILE, n - lo);
    for (int i = tid; i < TILE; i += NT) s_dst[i] = ~0u;
    if (DEP && tid < NW) {
        s_erid[tid][0] = EDGE_NONE;
        s_erid[tid][1] = EDGE_NONE;
    }
    double xv[IPT][D], vv[IPT][D];
    uint32_t mt[IPT], dst[IPT], q[IPT];
    uint32_t bad = 0;
    const bool full = lo + TILE <= n;
    // the head of the tile's run table (in range: the table has TILE entries
    // per tile), loaded with the state rather than after the run indices
    uint32_t rd0 = 0u, ro0 = 0u;
    if (tid < RUN_HEAD) {
        rd0 = run_dest[lo + tid];
        ro0 = run_info[lo + tid];
    }
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int64_t p = base + 64 * j;
        const bool ok = full || p < n;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            xv[j][k] = ok ? P.x[k][p] : 0.0;
            vv[j][k] = ok ? P.v[k][p] : 0.0;
        }
        mt[j] = ok ? meta[p] : 0u;
    }
    if (tid < RUN_HEAD) {
        s_rd[tid] = rd0;
        s_ro[tid] = ro0 & 0xffffu;
    }
    __syncthreads();   // run head in LDS, s_dst cleared
    uint32_t miss = 0, rid[IPT];
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int64_t p = base + 64 * j;
        dst[j] = ~0u;
        q[j] = ~0u;
        rid[j] = 0u;
        if (full || p < n) {
            rid[j] = min(mt[j] & 0xffffu, (uint32_t)TILE - 1u);
            const uint32_t rank = mt[j] >> 16;
            const bool head = rid[j] < (uint32_t)RUN_HEAD;
            const uint32_t d = (head ? s_rd[rid[j]] : run_dest[lo + rid[j]]) + rank;
            dst[j] = (d < (uint32_t)n && rid[j] == (mt[j] & 0xffffu)) ? d : ~0u;
            const uint32_t qq = (head ? s_ro[rid[j]] : (run_info[lo + rid[j]] & 0xffffu)) + rank;
            q[j] = qq < (uint32_t)cnt ? qq : ~0u;
            if (q[j] == ~0u) dst[j] = ~0u;
            if (dst[j] == ~0u) miss = 1;
        }
    }
    // the state as the key pass pushed it: again here, or stored by it
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int64_t p = base + 64 * j;
        if (PUSHED || !(full || p < n)) continue;
        int ii = 0;
        if (MULTI) ii = inst_of(inst_start, t.n_inst, p);
        const DevInst &in = MULTI ? t.inst[ii] : in0;
        const double qmdt = (MULTI && qa) ? qa[ii] : qmdt0;
        const double dt = (MULTI && da) ? da[ii] : dt0;
        if constexpr (MOVE == MOVE_PUSH)
            push_one<D, SCHEME, REG, false, false>(t, in, P, lds, lds_n, xv[j], vv[j], qmdt, dt, p, bad);
        else if constexpr (!PUSHED)   // the artificial flops belong to the key pass's move only
            stream_one<D, SCHEME, REG, MOVE - 1, false>(t, in, lds, lds_n, xv[j], vv[j], dt, 0, bad);
    }
    if (miss) flag_status(t.status, PIC_DEV_RANGE);
#pragma unroll
    for (int j = 0; j < IPT; ++j)
        if (dst[j] != ~0u) {
            s_dst[q[j]] = dst[j];
            if (DEP) s_rid[q[j]] = (uint16_t)rid[j];
        }
    // the state columns (unrolled, so the registers are indexed by
    // constants), then the extra columns, two at a time
    auto write_out = [&](int c0, int ncol) {
#pragma unroll
        for (int g = 0; g < SC; ++g) {
            const int c = c0 + g;
            if (c >= ncol) break;
            const bool st = c < 2 * D;
            const bool wide = st || extra.bytes[c - 2 * D] == 8;
            void *o = st ? (void *)(c < D ? out.x[c] : out.v[c - D]) : extra.out[c - 2 * D];
#pragma unroll
            for (int i = 0; i < IPT; ++i) {
                const int qq = tid + i * NT;
                if (qq >= cnt) break;
                const uint32_t d = s_dst[qq];
                if (d == ~0u) continue;
                if (wide) ((uint64_t *)o)[d] = s_val[g][qq];
                else ((uint32_t *)o)[d] = (uint32_t)s_val[g][qq];
            }
        }
    };
#pragma unroll
    for (int c0 = 0; c0 < 2 * D; c0 += SC) {
#pragma unroll
        for (int g = 0; g < SC; ++g) {
            const int c = c0 + g;
#pragma unroll
            for (int j = 0; j < IPT; ++j)
                if (dst[j] != ~0u) s_val[g][q[j]] = __double_as_longlong(c < D ? xv[j][c] : vv[j][c - D]);
        }
        __syncthreads();
        if constexpr (DEP) {
            if (c0 == 0)
                emit_deposit<D, SCHEME, TILE, NT, NSD>(in0, s_val, s_rid, s_edge, s_erid, lo, cnt, run_info, run_pos,
                                                       run_part);
            else if (c0 == 2 && tid < NW)
                emit_edges<NW, NSD>(s_edge, s_erid, lo, run_pos, run_part, t.status);
        }
        write_out(c0, 2 * D);
        __syncthreads();
    }
    const int ncol = 2 * D + extra.n;
    for (int c0 = 2 * D; c0 < ncol; c0 += SC) {
#pragma unroll
        for (int g = 0; g < SC; ++g) {
            const int c = c0 + g;
            if (c >= ncol) break;
            const int e = c - 2 * D;
            const bool wide = extra.bytes[e] == 8;
#pragma unroll
            for (int j = 0; j < IPT; ++j)
                if (dst[j] != ~0u)
                    s_val[g][q[j]] = wide ? ((const uint64_t *)extra.in[e])[base + 64 * j]
                                          : (uint64_t)((const uint32_t *)extra.in[e])[base + 64 * j];
        }
        __syncthreads();
        write_out(c0, ncol);
        __syncthreads();
    }
}

// Per bin: the sum of its runs' partials (stayers' runs of all tiles in tile
// order, then arrivals' runs in tile order: the runs' order in the output),
// the per-bin partials k_deposit_vertices sums per vertex.
template <int NS>
__global__ __launch_bounds__(256) void k_deposit_runs(const uint32_t *list_off, int64_t n_bins,
                                                      const double *run_part, double *partial) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < n_bins; b += stride) {
        const uint32_t r0 = list_off[2 * b], r1 = list_off[2 * b + 2];
        double acc[NS];
#pragma unroll
        for (int c = 0; c < NS; ++c) acc[c] = 0.0;
        for (uint32_t r = r0; r < r1; ++r)
#pragma unroll
            for (int c = 0; c < NS; ++c) acc[c] = __dadd_rn(acc[c], run_part[(int64_t)r * NS + c]);
#pragma unroll
        for (int c = 0; c < NS; ++c) partial[b * NS + c] = acc[c];
    }
}

// ----------------------------------------------------------------- launchers

struct StepArgs {
    uint32_t *zero;   // per-call counters, cleared by the key pass
    int64_t n_zero;
    F64Ptrs P, out;
    int64_t n;
    double qmdt, dt;
    const double *qa, *da;
    const int64_t *inst_start, *old_start;
    uint32_t n_bins;
    void *stats;      // nullable pic_rebin_stats record
    bool deposit;     // the writing pass deposits (2D regular single trees, uniform charge)
    int flops;        // free streaming: artificial flops per move (key pass)
    int ipt;          // particles per thread of a tile (step_ipt_of)
};

#define PIC_EMIT_AS(NT, DEP, EMOVE)                                                                           \
    PIC_LAUNCH("step_emit", (k_step_emit<D, SCH, REG, MULTI, TILE, NT, DEP, EMOVE>), dim3(tiles), dim3(NT), 0, s,   \
               t->dt,                                                                                               \
               t->inst0, a.P, a.n, a.qmdt, a.dt, a.qa, a.da, a.inst_start, (const uint32_t *)sc.meta,          \
               (const uint32_t *)sc.run_dest, (const uint32_t *)sc.run_info, (const uint32_t *)sc.run_pos,      \
               sc.run_part, a.out, extra, t->tune.xcd_tiles)
// the writing pass moves again, or only moves records the key pass stored
#define PIC_EMIT(NT, DEP)                                                                                     \
    do {                                                                                                      \
        if (stored) PIC_EMIT_AS(NT, DEP, MOVE_STORED);                                                        \
        else PIC_EMIT_AS(NT, DEP, MOVE);                                                                      \
    } while (0)

template <int D, int SCH, bool REG, bool MULTI, int TILE, int MOVE = MOVE_PUSH>
static void launch_step_passes(const pic_tree *t, const StepArgs &a, const RebinScratch &sc, const Cols &extra,
                               int64_t *new_start, hipStream_t s) {
    const int64_t tiles = (a.n + TILE - 1) / TILE;
    // the fused key+rank kernel pushes only; a streaming step takes the key
    // and ranking passes.  By default (step_fuse 2) 2D regular single trees
    // take it for PIT, unless the key pass is to store the pushed state.
    const bool fuse_auto = D == 2 && REG && !MULTI && SCH == PIC_PIT && t->tune.key_stores != 1;
    const bool fuse = (t->tune.step_fuse == 1 || (t->tune.step_fuse == 2 && fuse_auto)) && MOVE == MOVE_PUSH &&
                      TILE <= 2048;
    // the key pass stores the moved state (the fused key+rank kernel does not)
    const bool stored = t->tune.key_stores == 1 && !fuse;
    if (a.n > 0 && fuse) {
        // counters cleared first; the key pass and the ranking are one kernel
        launch_prep(a.zero, a.n_zero, nullptr, a.n_bins, a.n, TILE, sc, s);
        launch_keyrank(t, SCH, a.P, a.n, a.qmdt, a.dt, a.qa, a.da, a.inst_start, a.old_start, a.n_bins, TILE, sc,
                       a.stats ? sc.keys : nullptr, s);
        if (a.stats) (void)launch_rebin_stats(t, SCH, a.old_start, sc.keys, 1, a.n, a.stats, s);
    } else if (a.n > 0) {
        PIC_LAUNCH("step_key", (k_step_key<D, SCH, REG, MULTI, MOVE>), dim3(grid_for(a.n, 256, 1 << 20)), dim3(256), 0,
                   s, t->dt, t->inst0, a.P, a.n, a.qmdt, a.dt, a.qa, a.da, a.inst_start, a.old_start, a.n_bins,
                   sc.keys, a.zero, a.n_zero, stored ? 1 : 0, a.flops);
        if (a.stats) (void)launch_rebin_stats(t, SCH, a.old_start, sc.keys, 1, a.n, a.stats, s);
        launch_group(sc.keys, a.n, TILE, t->tune.group_match != 0, sc, s);
    }
    launch_step_middle(t, a.n, a.n_bins, sc, new_start, s);
    if (a.n == 0) return;
    if constexpr (D == 2 && REG && !MULTI && MOVE == MOVE_PUSH && TILE <= 2048) {
        if (a.deposit) {
            if (t->tune.emit_threads == 512) PIC_EMIT(512, true);
            else PIC_EMIT(1024, true);
            return;
        }
    }
    if (t->tune.emit_threads == 512) PIC_EMIT(512, false);
    else PIC_EMIT(1024, false);
}

template <int D, int SCH>
static void launch_step_shape(const pic_tree *t, const StepArgs &a, const RebinScratch &sc, const Cols &extra,
                              int64_t *new_start, hipStream_t s) {
    const bool multi = t->n_inst > 1, reg = t->reg_kernels != 0;
    const int ipt = a.ipt;
#define PIC_STEP_TILE(REG, MULTI)                                                                            \
    do {                                                                                                     \
        if (ipt == 4) launch_step_passes<D, SCH, REG, MULTI, 1024>(t, a, sc, extra, new_start, s);          \
        else if (ipt == 16) launch_step_passes<D, SCH, REG, MULTI, 4096>(t, a, sc, extra, new_start, s);    \
        else launch_step_passes<D, SCH, REG, MULTI, 2048>(t, a, sc, extra, new_start, s);                   \
    } while (0)
    if (multi) {
        if (reg) PIC_STEP_TILE(true, true); else PIC_STEP_TILE(false, true);
    } else {
        if (reg) PIC_STEP_TILE(true, false); else PIC_STEP_TILE(false, false);
    }
#undef PIC_STEP_TILE
}

hipError_t launch_step(const pic_tree *t, int scheme, pic_particles *in, const int64_t *old_start,
                       const double *const *E, double qmdt, double dt, const pic_push_params *pp, const Cols &extra,
                       pic_particles *out, int64_t *new_start, int q_col, double q_uniform, double *rho,
                       void *scratch, size_t scratch_bytes, void *stats, hipStream_t s) {
    const int64_t n = in->n;
    const int64_t n_bins = n_bins_of(t, scheme);
    const int ipt = step_ipt_of(t, n, n_bins), tile = RB_THREADS * ipt;
    const int ns = scheme == PIC_PIT ? 4 : 9;   // 2D deposit slots per run
    const RebinLayout L = rebin_layout(n, n_bins, tile, t->dim == 2 && tile <= 2048 ? ns : 0);
    if (scratch_bytes < L.total || scratch_bytes < deposit_scratch_bytes(t, scheme)) return hipErrorInvalidValue;
    char *base = (char *)scratch;
    const RebinScratch sc = bind_scratch(L, base);
    // the fused step's per-call counters: key_cn, the scan state and ticket,
    // the linked run lists' heads (contiguous in the layout)
    const int64_t zero_words = (int64_t)((L.key_base - L.key_cn) / 4);
    StepArgs a;
    a.zero = (uint32_t *)(base + L.key_cn);
    a.n_zero = zero_words;
    // the key pass clears the counters; with no particles there is none
    if (n == 0) launch_prep(a.zero, zero_words, nullptr, n_bins, n, tile, sc, s);
    a.P = make_ptrs(t, in, E, nullptr);
    a.out = make_ptrs(t, out, nullptr, nullptr);
    a.n = n;
    a.qmdt = qmdt;
    a.dt = dt;
    a.qa = pp ? pp->qmdt_dev : nullptr;
    a.da = pp ? pp->dt_dev : nullptr;
    a.inst_start = in->inst_start_dev;
    a.old_start = old_start;
    a.n_bins = (uint32_t)n_bins;
    a.stats = stats;
    // the writing pass deposits: on request, or by default for PIT (for
    // PIDT its nine-slot stencil costs the writing pass more than it saves)
    const bool dep_knob = t->tune.emit_deposit == 1 || (t->tune.emit_deposit == 2 && scheme == PIC_PIT);
    a.deposit = t->dim == 2 && t->reg_kernels && t->n_inst == 1 && q_col < 0 && dep_knob && tile <= 2048;
    a.flops = 0;
    a.ipt = ipt;
    if (t->dim == 2) {
        if (scheme == PIC_PIT) launch_step_shape<2, 0>(t, a, sc, extra, new_start, s);
        else launch_step_shape<2, 1>(t, a, sc, extra, new_start, s);
    } else {
        if (scheme == PIC_PIT) launch_step_shape<3, 0>(t, a, sc, extra, new_start, s);
        else launch_step_shape<3, 1>(t, a, sc, extra, new_start, s);
    }
    const double *q = q_col >= 0 ? (const double *)extra.out[q_col] : nullptr;
    if (!a.deposit || n == 0) return launch_deposit(t, scheme, out, new_start, q, q_uniform, rho, scratch, scratch_bytes, s);
    // the writing pass left one partial per run: sum them per bin, then per vertex
    double *partial = (double *)(base + L.bin_part);
    const dim3 g(grid_for(n_bins, 256, 1 << 16)), b(256);
    if (ns == 4) PIC_LAUNCH("deposit_runs", k_deposit_runs<4>, g, b, 0, s, (const uint32_t *)sc.list_off, n_bins,
                            (const double *)sc.run_part, partial);
    else PIC_LAUNCH("deposit_runs", k_deposit_runs<9>, g, b, 0, s, (const uint32_t *)sc.list_off, n_bins,
                    (const double *)sc.run_part, partial);
    launch_deposit_vertices(t, scheme, true, partial, false, q_uniform, rho, s);
    return hipGetLastError();
}

// The fused form of the particle-handling benchmark's step (single trees):
// the key pass streams every particle (with the artificial flops) and keys
// it, the ranking, scan and placement as in pic_step, the writing pass
// streams it again without the flops; no deposit.
template <int D, int SCH, int MOVE>
static void launch_stream_shape(const pic_tree *t, const StepArgs &a, const RebinScratch &sc, const Cols &extra,
                                int64_t *new_start, hipStream_t s) {
    const bool reg = t->reg_kernels != 0;
    const int ipt = a.ipt;
    if (reg) {
        if (ipt == 4) launch_step_passes<D, SCH, true, false, 1024, MOVE>(t, a, sc, extra, new_start, s);
        else if (ipt == 16) launch_step_passes<D, SCH, true, false, 4096, MOVE>(t, a, sc, extra, new_start, s);
        else launch_step_passes<D, SCH, true, false, 2048, MOVE>(t, a, sc, extra, new_start, s);
    } else {
        if (ipt == 4) launch_step_passes<D, SCH, false, false, 1024, MOVE>(t, a, sc, extra, new_start, s);
        else if (ipt == 16) launch_step_passes<D, SCH, false, false, 4096, MOVE>(t, a, sc, extra, new_start, s);
        else launch_step_passes<D, SCH, false, false, 2048, MOVE>(t, a, sc, extra, new_start, s);
    }
}

template <int D, int SCH>
static void launch_stream_bc(const pic_tree *t, int boundary, const StepArgs &a, const RebinScratch &sc,
                             const Cols &extra, int64_t *new_start, hipStream_t s) {
    if (boundary == PIC_PERIODIC) launch_stream_shape<D, SCH, MOVE_STREAM_PERIODIC>(t, a, sc, extra, new_start, s);
    else launch_stream_shape<D, SCH, MOVE_STREAM_REFLECTING>(t, a, sc, extra, new_start, s);
}

hipError_t launch_stream_step(const pic_tree *t, int scheme, pic_particles *in, const int64_t *old_start, double dt,
                              int boundary, int flops, const Cols &extra, pic_particles *out, int64_t *new_start,
                              void *scratch, size_t scratch_bytes, void *stats, hipStream_t s) {
    const int64_t n = in->n;
    const int64_t n_bins = n_bins_of(t, scheme);
    const int ipt = step_ipt_of(t, n, n_bins), tile = RB_THREADS * ipt;
    const int ns = scheme == PIC_PIT ? 4 : 9;
    const RebinLayout L = rebin_layout(n, n_bins, tile, t->dim == 2 && tile <= 2048 ? ns : 0);   // as pic_step
    if (scratch_bytes < L.total) return hipErrorInvalidValue;
    char *base = (char *)scratch;
    const RebinScratch sc = bind_scratch(L, base);
    const int64_t zero_words = (int64_t)((L.key_base - L.key_cn) / 4);
    StepArgs a;
    a.zero = (uint32_t *)(base + L.key_cn);
    a.n_zero = zero_words;
    if (n == 0) launch_prep(a.zero, zero_words, nullptr, n_bins, n, tile, sc, s);
    a.P = make_ptrs(t, in, nullptr, nullptr);
    a.out = make_ptrs(t, out, nullptr, nullptr);
    a.n = n;
    a.qmdt = 0.0;
    a.dt = dt;
    a.qa = nullptr;
    a.da = nullptr;
    a.inst_start = in->inst_start_dev;
    a.old_start = old_start;
    a.n_bins = (uint32_t)n_bins;
    a.stats = stats;
    a.deposit = false;
    a.flops = flops;
    a.ipt = ipt;
    if (t->dim == 2) {
        if (scheme == PIC_PIT) launch_stream_bc<2, 0>(t, boundary, a, sc, extra, new_start, s);
        else launch_stream_bc<2, 1>(t, boundary, a, sc, extra, new_start, s);
    } else {
        if (scheme == PIC_PIT) launch_stream_bc<3, 0>(t, boundary, a, sc, extra, new_start, s);
        else launch_stream_bc<3, 1>(t, boundary, a, sc, extra, new_start, s);
    }
    return hipGetLastError();
}

}  // namespace pic
