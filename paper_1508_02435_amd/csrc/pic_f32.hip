// pic_f32.hip -- the FP32 offset form: gather + push, the fused step's key
// and emit passes, the deposit with compensated per-bin sums, and the
// conversions between the FP64 and FP32 forms.
#include <hip/hip_runtime.h>

#include "pic_launch.h"

namespace pic {

// ------------------------------------------------------- FP32 offset form
//
// State per particle: off[k] in [0,1), the offset inside its finest cell in
// cell widths, and u[k], the velocity in finest cells per step (u = v dt 3^L).
// The cell itself is implicit in the particle's bin (regular instances: the
// leaf for PIT; for PIDT the owner vertex and the half of the offset).  The
// push moves the cell by the integer floor(off + u), exactly, and keeps the
// fraction in FP32, so bins stay integer-exact while positions carry FP32
// rounding.

struct F32Ptrs {
    float *off[3];
    float *u[3];
    const double *E[3];
};

// Lattice coordinates of lin = c0 + S c1 (+ S^2 c2), S = 3^L.
template <int D>
__device__ __forceinline__ void unlinear(uint32_t lin, int L, uint32_t S, uint32_t (&c)[D]) {
#pragma unroll
    for (int k = 0; k < D - 1; ++k) {
        const uint32_t q = div_pow3(lin, L);
        c[k] = lin - q * S;
        lin = q;
    }
    c[D - 1] = lin;
}

// Forest-wide bin -> instance-local rank, clamped (with a flag) for bins
// outside the instance.
template <int SCHEME>
__device__ __forceinline__ uint32_t local_rank(const DevInst &in, uint32_t bin, uint32_t &bad) {
    const uint32_t off = (uint32_t)(SCHEME == PIC_PIT ? in.leaf_off : in.pidt_off);
    const uint32_t cnt = (uint32_t)(SCHEME == PIC_PIT ? in.n_leaves : in.n_pidt);
    const uint32_t r = bin - off;
    if (r >= cnt) {
        bad |= PIC_DEV_RANGE;
        return 0u;
    }
    return r;
}

// Finest cell of a particle of a regular instance from its bin and offsets.
template <int D, int SCHEME>
__device__ __forceinline__ void cell_of(const DevTree &t, const DevInst &in, uint32_t rank, const float (&o)[D],
                                        uint32_t (&c)[D]) {
    const uint32_t S = (uint32_t)in.S;
    unlinear<D>(ld_const(t.cell_tab, (uint32_t)in.ptab + rank), in.L, S, c);
    if (SCHEME == PIC_PIDT) {
        const uint32_t half = (S - 1u) >> 1;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            uint32_t J = c[k] + S - half;             // back from the shifted lattice
            J = J >= S ? J - S : J;
            c[k] = o[k] >= 0.5f ? (J == 0u ? S - 1u : J - 1u) : J;
        }
    }
}

// Bin of a regular-instance particle in cell c with offsets o: the leaf, or
// the nearest corner (ties up) on the shifted lattice.
template <int D, int SCHEME>
__device__ __forceinline__ uint32_t bin_f32(const DevTree &t, const DevInst &in, const uint32_t (&c)[D],
                                            const float (&o)[D]) {
    if (SCHEME == PIC_PIT) return (uint32_t)in.leaf_off + regular_rank<D, true>(t, in, c);
    const uint32_t S = (uint32_t)in.S, half = (S - 1u) >> 1;
    uint32_t j[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        uint32_t J = c[k] + (o[k] >= 0.5f ? 1u : 0u) + half;
        j[k] = J >= S ? J - S : J;
    }
    return (uint32_t)in.pidt_off + regular_rank<D, true>(t, in, j);
}

// Cell coordinate moved by an integer amount d (any size), periodically.
__device__ __forceinline__ uint32_t wrap_shift(uint32_t c, float d, uint32_t S) {
    if (d >= 0.0f && d < (float)S) {
        const uint32_t r = c + (uint32_t)d;
        return r >= S ? r - S : r;
    }
    int64_t v = ((int64_t)c + (int64_t)d) % (int64_t)S;
    return (uint32_t)(v < 0 ? v + (int64_t)S : v);
}

// Gather + push of one particle in the FP32 form; returns the new bin.
template <int D, int SCHEME>
__device__ __forceinline__ uint32_t push_f32(const DevTree &t, const DevInst &in, const F32Ptrs &P,
                                             uint32_t (&c)[D], float (&o)[D], float (&u)[D], float kick,
                                             uint32_t &bad) {
    const uint32_t S = (uint32_t)in.S;
    uint32_t stride = 1, v0 = (uint32_t)in.vtx_off, step[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if (!(o[k] >= 0.0f && o[k] < 1.0f)) bad |= (o[k] == o[k]) ? PIC_DEV_RANGE : PIC_DEV_NONFINITE;
        if (!(u[k] - u[k] == 0.0f)) bad |= PIC_DEV_NONFINITE;
        v0 += __umul24(c[k], stride);
        step[k] = c[k] + 1u == S ? stride - __umul24(S, stride) : stride;
        stride = __umul24(stride, S);
    }
    uint32_t vid[1 << D];
#pragma unroll
    for (int cc = 0; cc < (1 << D); ++cc) {
        uint32_t v = v0;
#pragma unroll
        for (int k = 0; k < D; ++k)
            if ((cc >> k) & 1) v += step[k];
        vid[cc] = v;
    }
    float f[D], g[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        f[k] = fminf(fmaxf(o[k], 0.0f), 1.0f);      // malformed offsets (flagged) stay inside the cell
        g[k] = 1.0f - f[k];
    }
    float w[1 << D];
#pragma unroll
    for (int cc = 0; cc < (1 << D); ++cc) {
        float wc = (cc & 1) ? f[0] : g[0];
#pragma unroll
        for (int k = 1; k < D; ++k) wc *= ((cc >> k) & 1) ? f[k] : g[k];
        w[cc] = wc;
    }
    // corner field: scalar loads for the lanes sharing the first pending
    // lane's cell (field_passes passes), per-lane loads for the rest
    float Ec[1 << D][D];
    uint64_t pend = __ballot(1);
    const uint32_t lane = __lane_id();
#pragma unroll
    for (int it = 0; it < field_passes<D, SCHEME>(); ++it) {
        if (!pend) break;
        const int l = __builtin_ctzll(pend);
        const uint32_t v0u = (uint32_t)__builtin_amdgcn_readlane((int)vid[0], l);
        const bool mine = vid[0] == v0u;
        pend &= ~__ballot(mine);
        uint32_t vu[1 << D];
#pragma unroll
        for (int cc = 0; cc < (1 << D); ++cc) vu[cc] = (uint32_t)__builtin_amdgcn_readlane((int)vid[cc], l);
#pragma unroll
        for (int cc = 0; cc < (1 << D); ++cc)
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const float eu = (float)ld_const(P.E[j], vu[cc]);
                if (mine) Ec[cc][j] = eu;
            }
    }
    if ((pend >> lane) & 1ull) {
#pragma unroll
        for (int cc = 0; cc < (1 << D); ++cc)
#pragma unroll
            for (int j = 0; j < D; ++j) Ec[cc][j] = (float)ld_off(P.E[j], vid[cc]);
    }
#pragma unroll
    for (int j = 0; j < D; ++j) {
        float e = w[0] * Ec[0][j];
#pragma unroll
        for (int cc = 1; cc < (1 << D); ++cc) e += w[cc] * Ec[cc][j];
        const float uj = u[j] + kick * e;
        const float tp = f[j] + uj;
        float fl = floorf(tp);
        float no = tp - fl;
        if (no >= 1.0f) {                           // tiny negative tp: the fraction rounds up to 1
            no = 0.0f;
            fl += 1.0f;
        }
        if (!(fabsf(fl) < 1073741824.0f)) {         // non-finite or absurd displacement
            bad |= (tp == tp) ? PIC_DEV_RANGE : PIC_DEV_NONFINITE;
            fl = 0.0f;
            no = 0.0f;
        }
        c[j] = wrap_shift(c[j], fl, S);
        o[j] = no;
        u[j] = uj;
    }
    return bin_f32<D, SCHEME>(t, in, c, o);
}

// Segment of sorted offsets holding slot p: the largest b in [lo, hi] with
// start[b] <= p.
__device__ __forceinline__ uint32_t segment_of(const int64_t *start, uint32_t lo, uint32_t hi, int64_t p) {
    while (lo < hi) {
        const uint32_t m = (lo + hi + 1u) >> 1;
        if (start[m] <= p) lo = m;
        else hi = m - 1u;
    }
    return lo;
}

// Old bin of slot p of a sorted set: a binary search over the segment
// offsets, narrowed to the slot's tile when tile bounds are at hand.
__device__ __forceinline__ uint32_t old_bin_of(const int64_t *start, uint32_t n_bins, const uint32_t *tile_bin,
                                               int tile, int64_t p) {
    uint32_t lo = 0, hi = n_bins - 1u;
    if (tile_bin) {
        const int64_t tl = p / tile;
        lo = min(tile_bin[2 * tl], n_bins - 1u);
        hi = min(max(tile_bin[2 * tl + 1], lo + 1u), n_bins) - 1u;
    }
    return segment_of(start, lo, hi, p);
}

template <int D, int SCHEME, bool MULTI>
__global__ __launch_bounds__(256) void k_gather_push_f32(DevTree t, DevInst in0, F32Ptrs P, int64_t n,
                                                         double qmdt0, double dt0, const double *qa,
                                                         const double *da, const int64_t *inst_start,
                                                         const int64_t *bin_start, uint32_t n_bins,
                                                         const uint32_t *tile_bin, int tile, uint32_t *bin_out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        int ii = 0;
        if (MULTI) ii = inst_of(inst_start, t.n_inst, p);
        const DevInst &in = MULTI ? t.inst[ii] : in0;
        const double qmdt = (MULTI && qa) ? qa[ii] : qmdt0;
        const double dt = (MULTI && da) ? da[ii] : dt0;
        const float kick = (float)(qmdt * dt * in.Sd);
        uint32_t bad = 0;
        float o[D], u[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            o[k] = P.off[k][p];
            u[k] = P.u[k][p];
        }
        const uint32_t ob = old_bin_of(bin_start, n_bins, tile_bin, tile, p);
        uint32_t c[D];
        cell_of<D, SCHEME>(t, in, local_rank<SCHEME>(in, ob, bad), o, c);
        const uint32_t nb = push_f32<D, SCHEME>(t, in, P, c, o, u, kick, bad);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            P.off[k][p] = o[k];
            P.u[k][p] = u[k];
        }
        bin_out[p] = nb;
        if (bad) flag_status(t.status, bad);
    }
}

// Old bin of slot p with the wavefront's help: its slots are consecutive, so
// the first pending lane's bin is found once (scalar loads) and the lanes in
// it and in the next two bins are served from scalar loads of their bounds;
// lanes left search on their own.
__device__ __forceinline__ uint32_t old_bin_wave(const int64_t *start, uint32_t n_bins, const uint32_t *tile_bin,
                                                 int tile, int64_t p, const uint32_t *wave_bin) {
    uint64_t pend = __ballot(1);
    const uint32_t lane = __lane_id();
    const int l = __builtin_ctzll(pend);
    const int64_t pu = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)p, l)) |
                                 ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)p >> 32), l)
                                  << 32));
    uint32_t lo = 0, hi = n_bins - 1u;
    if (wave_bin) {
        // the bin of the first slot of pu's group of 64: one load, no search
        lo = hi = min(ld_const(wave_bin, (uint32_t)(pu >> 6)), n_bins - 1u);
    } else if (tile_bin) {
        const int64_t tl = pu / tile;
        lo = min(ld_const(tile_bin, (uint32_t)(2 * tl)), n_bins - 1u);
        hi = min(max(ld_const(tile_bin, (uint32_t)(2 * tl + 1)), lo + 1u), n_bins) - 1u;
    }
    while (lo < hi) {
        const uint32_t m = (lo + hi + 1u) >> 1;
        if (ld_const(start, m) <= pu) lo = m;
        else hi = m - 1u;
    }
    uint32_t ob = 0, bu = lo;
#pragma unroll
    for (int it = 0; it < 3; ++it) {
        if (!pend || bu >= n_bins) break;
        const int64_t s0 = ld_const(start, bu), s1 = ld_const(start, bu + 1u);
        const bool mine = ((pend >> lane) & 1ull) && s0 <= p && p < s1;
        if (mine) ob = bu;
        pend &= ~__ballot(mine);
        ++bu;
    }
    if ((pend >> lane) & 1ull) ob = old_bin_of(start, n_bins, tile_bin, tile, p);
    return ob;
}

// FP32 form, key pass of pic_step: one particle per thread, pushed, its key
// 2*bin + arrived written out (a particle arrives iff its bin changes: the
// bin is implicit in the segment it is stored in); with `store` the pushed
// offsets and velocities go back to the input arrays in place.  Like the
// FP64 key pass it waits on chained loads, so single trees ask for six
// resident wavefronts per SIMD (72 registers in 3D).
template <int D, int SCHEME, bool MULTI>
__global__ __launch_bounds__(256, MULTI ? 4 : 6) void k_step_key_f32(DevTree t, DevInst in0, F32Ptrs P, int64_t n, double qmdt0,
                                                      double dt0, const double *qa, const double *da,
                                                      const int64_t *inst_start, const int64_t *bin_start,
                                                      uint32_t n_bins, const uint32_t *tile_bin, int tile,
                                                      uint32_t *key_out, const uint32_t *wave_bin, int store) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // as the FP64 key pass: the writing pass's XCD chunks walked backwards
    const bool one_pass = stride >= n;
    const int64_t b0 = one_pass ? xcd_tile_rev(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    for (int64_t p = b0 * blockDim.x + threadIdx.x; p < n; p += one_pass ? n : stride) {
        int ii = 0;
        if (MULTI) ii = inst_of(inst_start, t.n_inst, p);
        const DevInst &in = MULTI ? t.inst[ii] : in0;
        const double qmdt = (MULTI && qa) ? qa[ii] : qmdt0;
        const double dt = (MULTI && da) ? da[ii] : dt0;
        const float kick = (float)(qmdt * dt * in.Sd);
        uint32_t bad = 0;
        float o[D], u[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            o[k] = P.off[k][p];
            u[k] = P.u[k][p];
        }
        const uint32_t ob = old_bin_wave(bin_start, n_bins, tile_bin, tile, p, wave_bin);
        uint32_t c[D];
        cell_of<D, SCHEME>(t, in, local_rank<SCHEME>(in, ob, bad), o, c);
        uint32_t nb = push_f32<D, SCHEME>(t, in, P, c, o, u, kick, bad);
        if (nb >= n_bins) bad |= PIC_DEV_RANGE;
        nb = min(nb, n_bins - 1u);
        key_out[p] = 2u * nb + (nb == ob ? 0u : 1u);
        if (store) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                P.off[k][p] = o[k];
                P.u[k][p] = u[k];
            }
        }
        if (bad) flag_status(t.status, bad);
    }
}

// FP32 form, emit pass of pic_step: the state pushed again (or, with
// PUSHED, as the key pass stored it) is staged through LDS in tile-sorted
// order, one column at a time, and written run by run (as k_step_emit).  The
// moving-only form holds no push code, so it needs fewer registers and more
// blocks fit a CU.
template <int D, int SCHEME, bool MULTI, int TILE, int NT, bool PUSHED>
__global__ __launch_bounds__(NT) void k_step_emit_f32(DevTree t, DevInst in0, F32Ptrs P, int64_t n, double qmdt0,
                                                      double dt0, const double *qa, const double *da,
                                                      const int64_t *inst_start, const int64_t *bin_start,
                                                      uint32_t n_bins, const uint32_t *tile_bin,
                                                      const uint32_t *meta, const uint32_t *run_dest,
                                                      const uint32_t *run_info, F32Ptrs out, Cols extra, int xcd,
                                                      const uint32_t *wave_bin) {
    constexpr int IPT = TILE / NT;
    __shared__ uint64_t s_val[TILE];
    __shared__ uint32_t s_dst[TILE];
    __shared__ uint32_t s_rd[RUN_HEAD], s_ro[RUN_HEAD];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t lo = xcd_tile(blockIdx.x, gridDim.x, xcd) * TILE;
    const int64_t base = lo + (int64_t)w * 64 * IPT + lane;
    const int cnt = (int)min((int64_t)TILE, n - lo);
    for (int i = tid; i < TILE; i += NT) s_dst[i] = ~0u;
    float o[IPT][D], u[IPT][D];
    uint32_t mt[IPT], dst[IPT], q[IPT];
    uint32_t bad = 0, miss = 0;
    uint32_t rd0 = 0u, ro0 = 0u;
    if (tid < RUN_HEAD) {
        rd0 = run_dest[lo + tid];
        ro0 = run_info[lo + tid];
    }
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int64_t p = base + 64 * j;
        const bool ok = p < n;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            o[j][k] = ok ? P.off[k][p] : 0.0f;
            u[j][k] = ok ? P.u[k][p] : 0.0f;
        }
        mt[j] = ok ? meta[p] : 0u;
    }
    if (tid < RUN_HEAD) {
        s_rd[tid] = rd0;
        s_ro[tid] = ro0 & 0xffffu;
    }
    __syncthreads();   // run head in LDS, s_dst cleared
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int64_t p = base + 64 * j;
        dst[j] = ~0u;
        q[j] = ~0u;
        if (p < n) {
            const uint32_t rid = min(mt[j] & 0xffffu, (uint32_t)TILE - 1u), rank = mt[j] >> 16;
            const bool head = rid < (uint32_t)RUN_HEAD;
            const uint32_t d = (head ? s_rd[rid] : run_dest[lo + rid]) + rank;
            const uint32_t qq = (head ? s_ro[rid] : (run_info[lo + rid] & 0xffffu)) + rank;
            if (d < (uint32_t)n && qq < (uint32_t)cnt && rid == (mt[j] & 0xffffu)) {
                dst[j] = d;
                q[j] = qq;
            } else {
                miss = 1;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int64_t p = base + 64 * j;
        if (PUSHED || p >= n) continue;   // PUSHED: the key pass stored the state
        int ii = 0;
        if (MULTI) ii = inst_of(inst_start, t.n_inst, p);
        const DevInst &in = MULTI ? t.inst[ii] : in0;
        const double qmdt = (MULTI && qa) ? qa[ii] : qmdt0;
        const double dt = (MULTI && da) ? da[ii] : dt0;
        const float kick = (float)(qmdt * dt * in.Sd);
        const uint32_t ob = old_bin_wave(bin_start, n_bins, tile_bin, TILE, p, wave_bin);
        uint32_t c[D];
        cell_of<D, SCHEME>(t, in, local_rank<SCHEME>(in, ob, bad), o[j], c);
        push_f32<D, SCHEME>(t, in, P, c, o[j], u[j], kick, bad);
    }
    if (miss) flag_status(t.status, PIC_DEV_RANGE);
#pragma unroll
    for (int j = 0; j < IPT; ++j)
        if (dst[j] != ~0u) s_dst[q[j]] = dst[j];
    const int ncol = 2 * D + extra.n;
    for (int c = 0; c < ncol; ++c) {
        const bool st = c < 2 * D;
        const bool wide = !st && extra.bytes[c - 2 * D] == 8;
        if (st) {
#pragma unroll
            for (int j = 0; j < IPT; ++j)
                if (dst[j] != ~0u) s_val[q[j]] = __float_as_uint(c < D ? o[j][c] : u[j][c - D]);
        } else {
            const int e = c - 2 * D;
#pragma unroll
            for (int j = 0; j < IPT; ++j)
                if (dst[j] != ~0u)
                    s_val[q[j]] = wide ? ((const uint64_t *)extra.in[e])[base + 64 * j]
                                       : (uint64_t)((const uint32_t *)extra.in[e])[base + 64 * j];
        }
        __syncthreads();
        void *ob = st ? (void *)(c < D ? out.off[c] : out.u[c - D]) : extra.out[c - 2 * D];
#pragma unroll
        for (int i = 0; i < IPT; ++i) {
            const int qq = tid + i * NT;
            if (qq >= cnt) break;
            const uint32_t d = s_dst[qq];
            if (d == ~0u) continue;
            if (wide) ((uint64_t *)ob)[d] = s_val[qq];
            else ((uint32_t *)ob)[d] = (uint32_t)s_val[qq];
        }
        __syncthreads();
    }
}

// Deposit partials of the FP32 form: per bin, FP32 compensated (Kahan) sums
// per lane in particle order, then a fixed FP64 tree over the G lanes.
template <int D, int SCHEME, int G, int K>
__global__ __launch_bounds__(256) void k_deposit_bins_f32(DevTree t, DevInst in0, F32Ptrs P, int64_t n,
                                                          const int64_t *bin_start, int64_t n_bins, const double *q,
                                                          double *partial) {
    constexpr int NS = SCHEME == PIC_PIT ? (1 << D) : (D == 2 ? 9 : 27);
    const int lane = threadIdx.x & (G - 1);
    const int64_t groups = (int64_t)gridDim.x * (blockDim.x / G);
    for (int64_t b = (int64_t)blockIdx.x * (blockDim.x / G) + (threadIdx.x / G); b < n_bins; b += groups) {
        float s[NS], cmp[NS];
#pragma unroll
        for (int k = 0; k < NS; ++k) s[k] = cmp[k] = 0.0f;
        int64_t p0 = bin_start[b], p1 = bin_start[b + 1];
        if (p0 < 0 || p1 > n || p0 > p1) {
            if (lane == 0) flag_status(t.status, PIC_DEV_RANGE);
            p0 = p1 = 0;
        }
        for (int64_t base = p0; base < p1; base += G * K) {
            float os[K][D], qs[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int64_t p = base + lane + G * k;
                const bool ok = p < p1;
#pragma unroll
                for (int d = 0; d < D; ++d) os[k][d] = ok ? P.off[d][p] : 0.0f;
                qs[k] = (ok && q) ? (float)q[p] : 1.0f;
            }
#pragma unroll
            for (int k = 0; k < K; ++k) {
                if (base + lane + G * k >= p1) continue;
                float f[D], g[D];
#pragma unroll
                for (int d = 0; d < D; ++d) {
                    f[d] = os[k][d];
                    g[d] = 1.0f - f[d];
                }
                float term[NS];
                if (SCHEME == PIC_PIT) {
#pragma unroll
                    for (int cc = 0; cc < NS; ++cc) {
                        float wc = (cc & 1) ? f[0] : g[0];
#pragma unroll
                        for (int d = 1; d < D; ++d) wc *= ((cc >> d) & 1) ? f[d] : g[d];
                        term[cc] = wc;
                    }
                } else {
                    // owner above the particle's cell (offset >= 1/2): corners at
                    // stencil offsets {-1, 0}, else {0, +1}
                    float w3[D][3];
#pragma unroll
                    for (int d = 0; d < D; ++d) {
                        const bool up = f[d] >= 0.5f;
                        w3[d][0] = up ? g[d] : 0.0f;
                        w3[d][1] = up ? f[d] : g[d];
                        w3[d][2] = up ? 0.0f : f[d];
                    }
#pragma unroll
                    for (int sl = 0; sl < NS; ++sl) {
                        float wc = w3[0][sl % 3] * w3[1][(sl / 3) % 3];
                        if (D == 3) wc *= w3[D - 1][sl / 9];
                        term[sl] = wc;
                    }
                }
#pragma unroll
                for (int cc = 0; cc < NS; ++cc) {
                    const float y = (q ? qs[k] * term[cc] : term[cc]) - cmp[cc];
                    const float tt = s[cc] + y;
                    cmp[cc] = (tt - s[cc]) - y;
                    s[cc] = tt;
                }
            }
        }
        double acc[NS];
#pragma unroll
        for (int cc = 0; cc < NS; ++cc) acc[cc] = (double)s[cc] - (double)cmp[cc];
        group_sum<G, NS>(acc);
        if (lane == 0) {
#pragma unroll
            for (int cc = 0; cc < NS; ++cc) partial[b * NS + cc] = acc[cc];
        }
    }
}

// FP64 -> FP32 form: the cell from y = fl(x 3^L) as in the FP64 path,
// off = fl32(y - I) (the subtraction is exact), u = fl32(v dt 3^L).
template <int D, int SCHEME, bool MULTI>
__global__ __launch_bounds__(256) void k_to_f32(DevTree t, DevInst in0, F64Ptrs X, F32Ptrs P, int64_t n, double dt0,
                                                const double *da, const int64_t *inst_start, uint32_t *bin_out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        int ii = 0;
        if (MULTI) ii = inst_of(inst_start, t.n_inst, p);
        const DevInst &in = MULTI ? t.inst[ii] : in0;
        const double dt = (MULTI && da) ? da[ii] : dt0;
        const uint32_t S = (uint32_t)in.S;
        uint32_t bad = 0, c[D];
        float o[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const Axis ax = scale_axis(X.x[k][p], in.Sd, in.S, bad);
            uint32_t I = ax.T >> 1;
            float ok = (float)__dsub_rn(ax.y, (double)I);
            if (ok >= 1.0f) {
                ok = 0.0f;
                I = I + 1u == S ? 0u : I + 1u;
            }
            c[k] = I;
            o[k] = ok;
            P.off[k][p] = ok;
            P.u[k][p] = (float)(X.v[k][p] * dt * in.Sd);
        }
        bin_out[p] = bin_f32<D, SCHEME>(t, in, c, o);
        if (bad) flag_status(t.status, bad);
    }
}

// FP32 -> FP64 form of a sorted set: x = (c + off) / 3^L, v = u / (dt 3^L).
template <int D, int SCHEME, bool MULTI>
__global__ __launch_bounds__(256) void k_to_f64(DevTree t, DevInst in0, F64Ptrs X, F32Ptrs P, int64_t n, double dt0,
                                                const double *da, const int64_t *inst_start,
                                                const int64_t *bin_start, uint32_t n_bins) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        int ii = 0;
        if (MULTI) ii = inst_of(inst_start, t.n_inst, p);
        const DevInst &in = MULTI ? t.inst[ii] : in0;
        const double dt = (MULTI && da) ? da[ii] : dt0;
        uint32_t bad = 0, c[D];
        float o[D];
#pragma unroll
        for (int k = 0; k < D; ++k) o[k] = P.off[k][p];
        const uint32_t ob = segment_of(bin_start, 0u, n_bins - 1u, p);
        cell_of<D, SCHEME>(t, in, local_rank<SCHEME>(in, ob, bad), o, c);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            double x = ((double)c[k] + (double)o[k]) / in.Sd;
            if (x >= 1.0) x -= 1.0;
            X.x[k][p] = x;
            X.v[k][p] = (double)P.u[k][p] / (dt * in.Sd);
        }
        if (bad) flag_status(t.status, bad);
    }
}

// ------------------------------------------------------ FP32 form launchers

static F32Ptrs make_f32(const pic_tree *t, const pic_particles *p, const double *const *E) {
    F32Ptrs P{};
    for (int k = 0; k < t->dim; ++k) {
        P.off[k] = p->off[k];
        P.u[k] = p->u[k];
        if (E) P.E[k] = E[k];
    }
    return P;
}

// dim x scheme x (single tree | forest) dispatch of a launcher template
#define PIC_SWITCH_DSM(FN, ...)                                                                          \
    do {                                                                                                 \
        const bool multi_ = t->n_inst > 1;                                                               \
        if (t->dim == 2) {                                                                               \
            if (scheme == PIC_PIT) { if (multi_) FN<2, 0, true>(__VA_ARGS__); else FN<2, 0, false>(__VA_ARGS__); } \
            else { if (multi_) FN<2, 1, true>(__VA_ARGS__); else FN<2, 1, false>(__VA_ARGS__); }         \
        } else {                                                                                         \
            if (scheme == PIC_PIT) { if (multi_) FN<3, 0, true>(__VA_ARGS__); else FN<3, 0, false>(__VA_ARGS__); } \
            else { if (multi_) FN<3, 1, true>(__VA_ARGS__); else FN<3, 1, false>(__VA_ARGS__); }         \
        }                                                                                                \
    } while (0)

template <int D, int SCH, bool MULTI>
static void gp_f32(const pic_tree *t, const F32Ptrs &P, int64_t n, double qmdt, double dt, const double *qa,
                   const double *da, const int64_t *inst_start, const int64_t *bin_start, uint32_t n_bins,
                   const uint32_t *tile_bin, int tile, uint32_t *bin, hipStream_t s) {
    PIC_LAUNCH("gather_push_f32", (k_gather_push_f32<D, SCH, MULTI>), dim3(grid_for(n, 256, 1 << 20)), dim3(256), 0,
               s, t->dt, t->inst0, P, n, qmdt, dt, qa, da, inst_start, bin_start, n_bins, tile_bin, tile, bin);
}

hipError_t launch_gather_push_f32(const pic_tree *t, int scheme, pic_particles *p, const double *const *E,
                                  double qmdt, double dt, const pic_push_params *pp, const int64_t *bin_start,
                                  const uint32_t *tile_bin, int tile, uint32_t *bin, hipStream_t s) {
    if (p->n == 0) return hipSuccess;
    const F32Ptrs P = make_f32(t, p, E);
    const double *qa = pp ? pp->qmdt_dev : nullptr;
    const double *da = pp ? pp->dt_dev : nullptr;
    const uint32_t n_bins = (uint32_t)n_bins_of(t, scheme);
    PIC_SWITCH_DSM(gp_f32, t, P, p->n, qmdt, dt, qa, da, p->inst_start_dev, bin_start, n_bins, tile_bin, tile, bin, s);
    return hipGetLastError();
}

template <int D, int SCH, bool MULTI>
static void dep_f32(const pic_tree *t, const F32Ptrs &P, int64_t n, const int64_t *bin_start, int64_t n_bins,
                    const double *q, double q_uniform, double *partial, double *rho, hipStream_t s) {
    const int64_t n_vtx = t->vtx_off.back();
    PIC_LAUNCH("deposit_bins_f32", (k_deposit_bins_f32<D, SCH, 64, 4>), dim3(grid_for(n_bins, 4, 1 << 18)), dim3(256),
               0, s, t->dt, t->inst0, P, n, bin_start, n_bins, q, partial);
    (void)n_vtx;
    launch_deposit_vertices(t, SCH, true, partial, q != nullptr, q_uniform, rho, s);
}

hipError_t launch_deposit_f32(const pic_tree *t, int scheme, const pic_particles *p, const int64_t *bin_start,
                              const double *q, double q_uniform, double *rho, void *scratch, size_t scratch_bytes,
                              hipStream_t s) {
    if (scratch_bytes < deposit_scratch_bytes(t, scheme)) return hipErrorInvalidValue;
    const F32Ptrs P = make_f32(t, p, nullptr);
    PIC_SWITCH_DSM(dep_f32, t, P, p->n, bin_start, n_bins_of(t, scheme), q, q_uniform, (double *)scratch, rho, s);
    return hipGetLastError();
}

template <int D, int SCH, bool MULTI>
static void conv(const pic_tree *t, bool to_f32, const F64Ptrs &X, const F32Ptrs &P, int64_t n, double dt,
                 const double *da, const int64_t *inst_start, const int64_t *bin_start, uint32_t *bin,
                 hipStream_t s) {
    const dim3 g(grid_for(n, 256, 1 << 20));
    if (to_f32)
        PIC_LAUNCH("to_f32", (k_to_f32<D, SCH, MULTI>), g, dim3(256), 0, s, t->dt, t->inst0, X, P, n, dt, da,
                   inst_start, bin);
    else
        PIC_LAUNCH("to_f64", (k_to_f64<D, SCH, MULTI>), g, dim3(256), 0, s, t->dt, t->inst0, X, P, n, dt, da,
                   inst_start, bin_start, (uint32_t)n_bins_of(t, SCH));
}

hipError_t launch_convert(const pic_tree *t, int scheme, int to_precision, pic_particles *p, double dt,
                          const pic_push_params *pp, const int64_t *bin_start, uint32_t *bin, hipStream_t s) {
    if (p->n == 0) return hipSuccess;
    const F64Ptrs X = make_ptrs(t, p, nullptr, nullptr);
    const F32Ptrs P = make_f32(t, p, nullptr);
    const double *da = pp ? pp->dt_dev : nullptr;
    PIC_SWITCH_DSM(conv, t, to_precision == PIC_F32_OFFSET, X, P, p->n, dt, da, p->inst_start_dev, bin_start, bin, s);
    return hipGetLastError();
}

size_t step_f32_scratch_bytes(const pic_tree *t, int64_t n, int scheme) {
    return std::max(rebin_scratch_bytes(t, n, scheme) + align256((size_t)n * 4), deposit_scratch_bytes(t, scheme));
}

// One FP32 step: gather + push in place on `in` (old bins from the tile
// bounds of the old order), stable re-bin of the FP32 columns into `out`,
// deposit on `out`.
template <int D, int SCH, bool MULTI>
static void step_passes_f32(const pic_tree *t, const F32Ptrs &P, const F32Ptrs &Q, int64_t n, double qmdt, double dt,
                            const double *qa, const double *da, const int64_t *inst_start, const int64_t *old_start,
                            uint32_t n_bins, const RebinScratch &sc, const Cols &extra, int64_t *new_start,
                            void *stats, int tile, hipStream_t s) {
    const int64_t tiles = (n + tile - 1) / tile;
    const int stored = t->tune.key_stores == 1 || (t->tune.key_stores == 2 && D == 3);
    PIC_LAUNCH("step_key_f32", (k_step_key_f32<D, SCH, MULTI>), dim3(grid_for(n, 256, 1 << 20)), dim3(256), 0, s,
               t->dt, t->inst0, P, n, qmdt, dt, qa, da, inst_start, old_start, n_bins, (const uint32_t *)sc.tile_bin,
               tile, sc.keys, (const uint32_t *)sc.wave_bin, stored);
    if (stats) (void)launch_rebin_stats(t, SCH, old_start, sc.keys, 1, n, stats, s);
    launch_group(sc.keys, n, tile, t->tune.group_match != 0, sc, s);
    launch_step_middle(t, n, n_bins, sc, new_start, s);
#define PIC_EMIT_F32(TILE, PUSHED)                                                                                 \
    PIC_LAUNCH("step_emit_f32", (k_step_emit_f32<D, SCH, MULTI, TILE, 1024, PUSHED>), dim3(tiles), dim3(1024), 0, s,  \
               t->dt, t->inst0, P, n, qmdt, dt, qa, da, inst_start, old_start, n_bins,                              \
               (const uint32_t *)sc.tile_bin, (const uint32_t *)sc.meta, (const uint32_t *)sc.run_dest,              \
               (const uint32_t *)sc.run_info, Q, extra, t->tune.xcd_tiles, (const uint32_t *)sc.wave_bin)
    if (tile == 4096) {
        if (stored) PIC_EMIT_F32(4096, true);
        else PIC_EMIT_F32(4096, false);
    } else {
        if (stored) PIC_EMIT_F32(2048, true);
        else PIC_EMIT_F32(2048, false);
    }
#undef PIC_EMIT_F32
}

hipError_t launch_step_f32(const pic_tree *t, int scheme, pic_particles *in, const int64_t *old_start,
                           const double *const *E, double qmdt, double dt, const pic_push_params *pp,
                           const Cols &extra, pic_particles *out, int64_t *new_start, int q_col, double q_uniform,
                           double *rho, void *scratch, size_t scratch_bytes, void *stats, hipStream_t s) {
    const int64_t n = in->n;
    const int64_t n_bins = n_bins_of(t, scheme);
    if (scratch_bytes < step_f32_scratch_bytes(t, n, scheme)) return hipErrorInvalidValue;
    if (n > 0) {
        // key, group, scan, place and emit passes, as the FP64 step; tiles of
        // 4096 where that step takes them (step_ipt_of), else 2048
        const int tile = step_ipt_of(t, n, n_bins) == 16 ? 4096 : 2048;
        const RebinLayout L = rebin_layout(n, n_bins, tile);
        char *base = (char *)scratch;
        const RebinScratch sc = bind_scratch(L, base);
        const int64_t zero_words = (int64_t)((L.key_base - L.key_cnt) / 4);
        launch_prep((uint32_t *)(base + L.key_cnt), zero_words, old_start, n_bins, n, tile, sc, s);
        const F32Ptrs P = make_f32(t, in, E), Q = make_f32(t, out, E);
        const double *qa = pp ? pp->qmdt_dev : nullptr;
        const double *da = pp ? pp->dt_dev : nullptr;
        PIC_SWITCH_DSM(step_passes_f32, t, P, Q, n, qmdt, dt, qa, da, in->inst_start_dev, old_start,
                       (uint32_t)n_bins, sc, extra, new_start, stats, tile, s);
        const double *q = q_col >= 0 ? (const double *)extra.out[q_col] : nullptr;
        return launch_deposit_f32(t, scheme, out, new_start, q, q_uniform, rho, scratch, scratch_bytes, s);
    }
    const size_t rb = rebin_scratch_bytes(t, n, scheme);
    char *base = (char *)scratch;
    uint32_t *bins = (uint32_t *)(base + rb);
    const int tile = RB_THREADS * t->tune.rebin_ipt;
    const RebinLayout L = rebin_layout(n, n_bins, tile);
    const RebinScratch sc = bind_scratch(L, base);
    if (n > 0) {
        launch_prep(nullptr, 0, old_start, n_bins, n, tile, sc, s);
        hipError_t e = launch_gather_push_f32(t, scheme, in, E, qmdt, dt, pp, old_start, sc.tile_bin, tile, bins, s);
        if (e != hipSuccess) return e;
    }
    Cols cols{};
    for (int k = 0; k < t->dim; ++k) {
        cols.in[cols.n] = in->off[k]; cols.out[cols.n] = out->off[k]; cols.bytes[cols.n++] = 4;
    }
    for (int k = 0; k < t->dim; ++k) {
        cols.in[cols.n] = in->u[k]; cols.out[cols.n] = out->u[k]; cols.bytes[cols.n++] = 4;
    }
    for (int c = 0; c < extra.n; ++c) {
        cols.in[cols.n] = extra.in[c]; cols.out[cols.n] = extra.out[c]; cols.bytes[cols.n++] = extra.bytes[c];
    }
    hipError_t e = launch_rebin(t, scheme, n, bins, old_start, cols, new_start, scratch, rb, s);
    if (e != hipSuccess) return e;
    const double *q = q_col >= 0 ? (const double *)extra.out[q_col] : nullptr;
    return launch_deposit_f32(t, scheme, out, new_start, q, q_uniform, rho, scratch, scratch_bytes, s);
}

}  // namespace pic
