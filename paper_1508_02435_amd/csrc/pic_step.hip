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

// Key pass: one particle per thread, pushed, its key
// 2*bin + arrived written out (the state itself is not).
template <int D, int SCHEME, bool REG, bool MULTI>
__global__ __launch_bounds__(256) void k_step_key(DevTree t, DevInst in0, F64Ptrs P, int64_t n, double qmdt0,
                                                  double dt0, const double *qa, const double *da,
                                                  const int64_t *inst_start, const int64_t *old_start,
                                                  uint32_t n_bins, uint32_t *key_out, uint32_t *zero,
                                                  int64_t n_zero) {
    __shared__ int32_t lds[REG ? 1 : PIC_LDS_NODES];
    const int lds_n = MULTI ? 0 : stage_nodes<REG>(t, in0, lds);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_zero; i += stride) zero[i] = 0u;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        int ii = 0;
        if (MULTI) ii = inst_of(inst_start, t.n_inst, p);
        const DevInst &in = MULTI ? t.inst[ii] : in0;
        const double qmdt = (MULTI && qa) ? qa[ii] : qmdt0;
        const double dt = (MULTI && da) ? da[ii] : dt0;
        uint32_t bad = 0;
        double xv[D], vv[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            xv[k] = P.x[k][p];
            vv[k] = P.v[k][p];
        }
        // finest cell of the old position (PIT on a regular instance: its bin)
        uint32_t cold = 0;
        if (SCHEME == PIC_PIT && REG) {
            uint32_t m = 1;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const double y = x_scaled(xv[k], in.Sd);
                cold += __umul24(min((uint32_t)max(y, 0.0), (uint32_t)in.S - 1u), m);
                m = __umul24(m, (uint32_t)in.S);
            }
        }
        uint32_t b = push_one<D, SCHEME, REG, false>(t, in, P, lds, lds_n, xv, vv, qmdt, dt, p, bad);
        if (b >= n_bins) bad |= PIC_DEV_RANGE;
        b = min(b, n_bins - 1);
        // A particle stays iff its slot lies in its new bin's old segment.
        // When the slot lies in the old segment of the bin of its old cell,
        // that is the case iff the two bins agree; the lanes of a wavefront
        // mostly share that cell, so its bin and segment come from scalar
        // loads.  Other lanes load the new bin's segment.
        bool stay = false, known = !old_start;
        if (SCHEME == PIC_PIT && REG && !MULTI && old_start) {
            uint64_t pend = __ballot(1);
#pragma unroll
            for (int it = 0; it < 2; ++it) {
                if (!pend) break;
                const uint32_t cu = (uint32_t)__builtin_amdgcn_readlane((int)cold, __builtin_ctzll(pend));
                const bool mine = cold == cu;
                pend &= ~__ballot(mine);
                const uint32_t ob = (uint32_t)in.leaf_off + ld_const(t.peano_tab, (uint32_t)in.ptab + cu);
                const int64_t s0 = ld_const(old_start, ob), s1 = ld_const(old_start, ob + 1u);
                if (mine && s0 <= p && p < s1) {
                    stay = b == ob;
                    known = true;
                }
            }
        }
        if (!known) stay = old_start[b] <= p && p < old_start[b + 1];
        key_out[p] = 2u * b + (stay ? 0u : 1u);
        if (bad) flag_status(t.status, bad);
    }
}

// Emit pass: slot p of tile T writes its pushed state to
// run_dest[T's run area + rid] + rank.  NT threads cover the TILE slots of a
// tile.  With STAGE the tile's records are first put in tile-local sorted
// order (runs one after the other, each run at its start from the run table)
// through LDS, STAGE columns at a time, so that a wavefront's stores cover
// consecutive destinations of a few runs instead of a few elements of each of
// many runs.
template <int D, int SCHEME, bool REG, bool MULTI, int TILE, int NT, int STAGE>
__global__ __launch_bounds__(NT) void k_step_emit(DevTree t, DevInst in0, F64Ptrs P, int64_t n, double qmdt0,
                                                  double dt0, const double *qa, const double *da,
                                                  const int64_t *inst_start, const uint32_t *meta,
                                                  const uint32_t *run_dest, const uint32_t *run_info, F64Ptrs out,
                                                  Cols extra, int xcd) {
    constexpr int IPT = TILE / NT;
    constexpr int NS = STAGE > 0 ? STAGE : 1;
    __shared__ int32_t lds[REG ? 1 : PIC_LDS_NODES];
    __shared__ uint64_t s_val[STAGE ? NS : 1][STAGE ? TILE : 1];
    __shared__ uint32_t s_dst[STAGE ? TILE : 1];
    __shared__ uint32_t s_rd[RUN_HEAD], s_ro[RUN_HEAD];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t lo = xcd_tile(blockIdx.x, gridDim.x, xcd) * TILE;
    const int lds_n = MULTI ? 0 : stage_nodes<REG>(t, in0, lds);
    const int64_t base = lo + (int64_t)w * 64 * IPT + lane;
    const int cnt = (int)min((int64_t)TILE, n - lo);
    if (STAGE)
        for (int i = tid; i < TILE; i += NT) s_dst[i] = ~0u;
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
    uint32_t miss = 0;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int64_t p = base + 64 * j;
        dst[j] = ~0u;
        q[j] = ~0u;
        if (full || p < n) {
            const uint32_t rid = min(mt[j] & 0xffffu, (uint32_t)TILE - 1u), rank = mt[j] >> 16;
            const bool head = rid < (uint32_t)RUN_HEAD;
            const uint32_t d = (head ? s_rd[rid] : run_dest[lo + rid]) + rank;
            dst[j] = (d < (uint32_t)n && rid == (mt[j] & 0xffffu)) ? d : ~0u;
            if (STAGE) {
                const uint32_t qq = (head ? s_ro[rid] : (run_info[lo + rid] & 0xffffu)) + rank;
                q[j] = qq < (uint32_t)cnt ? qq : ~0u;
                if (q[j] == ~0u) dst[j] = ~0u;
            }
            if (dst[j] == ~0u) miss = 1;
        }
    }
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int64_t p = base + 64 * j;
        if (!(full || p < n)) continue;
        int ii = 0;
        if (MULTI) ii = inst_of(inst_start, t.n_inst, p);
        const DevInst &in = MULTI ? t.inst[ii] : in0;
        const double qmdt = (MULTI && qa) ? qa[ii] : qmdt0;
        const double dt = (MULTI && da) ? da[ii] : dt0;
        push_one<D, SCHEME, REG, false, false>(t, in, P, lds, lds_n, xv[j], vv[j], qmdt, dt, p, bad);
    }
    if (miss) flag_status(t.status, PIC_DEV_RANGE);
    if (!STAGE) {
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            if (dst[j] == ~0u) continue;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                out.x[k][dst[j]] = xv[j][k];
                out.v[k][dst[j]] = vv[j][k];
            }
        }
        for (int c = 0; c < extra.n; ++c) {
            if (extra.bytes[c] == 8) {
                const uint64_t *src = (const uint64_t *)extra.in[c];
                uint64_t *o = (uint64_t *)extra.out[c];
                uint64_t v[IPT];
#pragma unroll
                for (int j = 0; j < IPT; ++j) v[j] = dst[j] != ~0u ? src[base + 64 * j] : 0u;
#pragma unroll
                for (int j = 0; j < IPT; ++j)
                    if (dst[j] != ~0u) o[dst[j]] = v[j];
            } else {
                const uint32_t *src = (const uint32_t *)extra.in[c];
                uint32_t *o = (uint32_t *)extra.out[c];
                uint32_t v[IPT];
#pragma unroll
                for (int j = 0; j < IPT; ++j) v[j] = dst[j] != ~0u ? src[base + 64 * j] : 0u;
#pragma unroll
                for (int j = 0; j < IPT; ++j)
                    if (dst[j] != ~0u) o[dst[j]] = v[j];
            }
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < IPT; ++j)
        if (dst[j] != ~0u) s_dst[q[j]] = dst[j];
    // the 2D state columns, then the extra columns, NS at a time
    const int ncol = 2 * D + extra.n;
    for (int c0 = 0; c0 < ncol; c0 += NS) {
#pragma unroll
        for (int g = 0; g < NS; ++g) {
            const int c = c0 + g;
            if (c >= ncol) break;
            if (c < 2 * D) {
#pragma unroll
                for (int j = 0; j < IPT; ++j)
                    if (dst[j] != ~0u) s_val[g][q[j]] = __double_as_longlong(c < D ? xv[j][c] : vv[j][c - D]);
            } else {
                const int e = c - 2 * D;
                const bool wide = extra.bytes[e] == 8;
#pragma unroll
                for (int j = 0; j < IPT; ++j)
                    if (dst[j] != ~0u)
                        s_val[g][q[j]] = wide ? ((const uint64_t *)extra.in[e])[base + 64 * j]
                                              : (uint64_t)((const uint32_t *)extra.in[e])[base + 64 * j];
            }
        }
        __syncthreads();
#pragma unroll
        for (int g = 0; g < NS; ++g) {
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
        __syncthreads();
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
};

#define PIC_EMIT(NT)                                                                                          \
    PIC_LAUNCH("step_emit", (k_step_emit<D, SCH, REG, MULTI, TILE, NT, 2>), dim3(tiles), dim3(NT), 0, s, t->dt, \
               t->inst0, a.P, a.n, a.qmdt, a.dt, a.qa, a.da, a.inst_start, (const uint32_t *)sc.meta,          \
               (const uint32_t *)sc.run_dest, (const uint32_t *)sc.run_info, a.out, extra, t->tune.xcd_tiles)

template <int D, int SCH, bool REG, bool MULTI, int TILE>
static void launch_step_passes(const pic_tree *t, const StepArgs &a, const RebinScratch &sc, const Cols &extra,
                               int64_t *new_start, hipStream_t s) {
    const int64_t tiles = (a.n + TILE - 1) / TILE;
    if (a.n > 0) {
        PIC_LAUNCH("step_key", (k_step_key<D, SCH, REG, MULTI>), dim3(grid_for(a.n, 256, 1 << 20)), dim3(256), 0, s,
                   t->dt, t->inst0, a.P, a.n, a.qmdt, a.dt, a.qa, a.da, a.inst_start, a.old_start, a.n_bins,
                   sc.keys, a.zero, a.n_zero);
        if (a.stats) (void)launch_rebin_stats(t, SCH, a.old_start, sc.keys, 1, a.n, a.stats, s);
        launch_group(sc.keys, a.n, TILE, sc, s);
    }
    launch_step_middle(t, a.n, a.n_bins, sc, new_start, s);
    if (a.n == 0) return;
    if (t->tune.emit_threads == 512) PIC_EMIT(512);
    else PIC_EMIT(1024);
}

template <int D, int SCH>
static void launch_step_shape(const pic_tree *t, const StepArgs &a, const RebinScratch &sc, const Cols &extra,
                              int64_t *new_start, hipStream_t s) {
    const bool multi = t->n_inst > 1, reg = t->reg_kernels != 0, small = t->tune.step_ipt == 4;
#define PIC_STEP_TILE(REG, MULTI)                                                                            \
    do {                                                                                                     \
        if (small) launch_step_passes<D, SCH, REG, MULTI, 1024>(t, a, sc, extra, new_start, s);             \
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
    const int tile = RB_THREADS * t->tune.step_ipt;
    const RebinLayout L = rebin_layout(n, n_bins, tile);
    if (scratch_bytes < L.total || scratch_bytes < deposit_scratch_bytes(t, scheme)) return hipErrorInvalidValue;
    char *base = (char *)scratch;
    const RebinScratch sc = bind_scratch(L, base);
    const int64_t zero_words = (int64_t)((L.key_base - L.key_cnt) / 4);
    StepArgs a;
    a.zero = (uint32_t *)(base + L.key_cnt);
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
    if (t->dim == 2) {
        if (scheme == PIC_PIT) launch_step_shape<2, 0>(t, a, sc, extra, new_start, s);
        else launch_step_shape<2, 1>(t, a, sc, extra, new_start, s);
    } else {
        if (scheme == PIC_PIT) launch_step_shape<3, 0>(t, a, sc, extra, new_start, s);
        else launch_step_shape<3, 1>(t, a, sc, extra, new_start, s);
    }
    const double *q = q_col >= 0 ? (const double *)extra.out[q_col] : nullptr;
    return launch_deposit(t, scheme, out, new_start, q, q_uniform, rho, scratch, scratch_bytes, s);
}

}  // namespace pic
