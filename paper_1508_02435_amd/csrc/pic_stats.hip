// pic_stats.hip -- re-bin statistics (paper Sec. 6.1: lifts per particle and
// time step).  In the paper's PIT a particle that leaves its leaf is lifted
// to the parent until a cell covers it and then dropped into the leaf that
// holds it, so a particle moving from leaf a to leaf b is lifted
// level(a) - level(c) times, c being the coarsest common ancestor of a and b
// ("n levels = n lifts").  The same count is taken in the dual tree for
// PIDT: dual cells of a k = 3 spacetree nest (Sec. 4.1), and on the lattice
// shifted by half the domain the dual cell of a level-l vertex b is the
// aligned level-l cell (b + (3^l - 1)/2) mod 3^l, so the common ancestor of
// two dual cells is found on those shifted coordinates.
//
// Per particle: old bin (the segment of the old offsets that holds its
// slot), new bin, mover flag, lift count, and the tunnel distance, the
// periodic max-norm distance between the old and the new bin's anchor (leaf
// corner or vertex position) in finest cells.  Integer counters only,
// reduced per wavefront and per block, then added to the caller's record
// with integer atomics, so the result does not depend on scheduling.
#include <hip/hip_runtime.h>

#include "pic_launch.h"

namespace pic {

// Bin holding slot p of a sorted set: the last b with start[b] <= p among
// non-empty segments (upper bound over start[1..n_bins]).
__device__ __forceinline__ uint32_t slot_bin(const int64_t *start, uint32_t n_bins, int64_t p) {
    uint32_t lo = 0, hi = n_bins;   // answer in [0, n_bins)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (start[mid] <= p) lo = mid; else hi = mid;
    }
    return lo;
}

// Anchor of a bin in finest units of its instance: the lower corner of a
// leaf (PIT), the vertex position (PIDT, `shifted` false) or the lower
// corner of the vertex's dual cell on the half-shifted lattice (`shifted`).
template <int D, int SCHEME>
__device__ __forceinline__ void bin_anchor(const DevTree &t, uint32_t b, int L, int lev, bool shifted,
                                           uint32_t (&A)[D]) {
    const uint32_t s = pow3_u32(L - lev), n_l = pow3_u32(lev);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        uint32_t a = SCHEME == PIC_PIT ? t.leaf_coord[(int64_t)b * D + k] : t.pidt_b[(int64_t)b * D + k];
        if (SCHEME == PIC_PIDT && shifted) {
            a += (n_l - 1u) >> 1;
            if (a >= n_l) a -= n_l;
        }
        A[k] = a * s;
    }
}

template <int D, int SCHEME>
__global__ __launch_bounds__(256) void k_rebin_stats(DevTree t, const int64_t *old_start, const uint32_t *bins,
                                                     int shift, int64_t n, uint32_t n_bins,
                                                     unsigned long long *out) {
    __shared__ unsigned long long s_acc[3 + PIC_STATS_LEVELS];   // movers, lifts, max, histogram
    const int tid = threadIdx.x, lane = tid & 63;
    for (int i = tid; i < 3 + PIC_STATS_LEVELS; i += blockDim.x) s_acc[i] = 0ull;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t bad = 0;
    for (int64_t p0 = (int64_t)blockIdx.x * blockDim.x; p0 < n; p0 += stride) {
        const int64_t p = p0 + tid;
        const bool live = p < n;
        bool mover = false;
        uint32_t lifts = 0, dist = 0;
        if (live) {
            uint32_t b1 = bins[p] >> shift;
            if (b1 >= n_bins) {
                bad |= PIC_DEV_RANGE;
                b1 = n_bins - 1;
            }
            const uint32_t b0 = slot_bin(old_start, n_bins, p);
            mover = b0 != b1;
            if (mover) {
                const int ii = t.n_inst > 1 ? (SCHEME == PIC_PIT ? t.leaf_inst[b0] : t.pidt_inst[b0]) : 0;
                const int ij = t.n_inst > 1 ? (SCHEME == PIC_PIT ? t.leaf_inst[b1] : t.pidt_inst[b1]) : 0;
                if (ii != ij) bad |= PIC_DEV_RANGE;
                const DevInst &in = t.inst[ii];
                const int L = in.L;
                const uint32_t S = (uint32_t)in.S;
                const int l0 = SCHEME == PIC_PIT ? t.leaf_level[b0] : t.pidt_level[b0];
                const int l1 = SCHEME == PIC_PIT ? t.leaf_level[b1] : t.pidt_level[b1];
                uint32_t A0[D], A1[D];
                bin_anchor<D, SCHEME>(t, b0, L, l0, false, A0);
                bin_anchor<D, SCHEME>(t, b1, L, l1, false, A1);
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    const uint32_t d = A0[k] > A1[k] ? A0[k] - A1[k] : A1[k] - A0[k];
                    dist = max(dist, min(d, S - d));
                }
                if (SCHEME == PIC_PIDT) {
                    bin_anchor<D, SCHEME>(t, b0, L, l0, true, A0);
                    bin_anchor<D, SCHEME>(t, b1, L, l1, true, A1);
                }
                int l = min(l0, l1);
                for (; l > 0; --l) {
                    bool same = true;
#pragma unroll
                    for (int k = 0; k < D; ++k) same &= div_pow3(A0[k], L - l) == div_pow3(A1[k], L - l);
                    if (same) break;
                }
                lifts = (uint32_t)(l0 - l);
            }
        }
        // wavefront reductions, then one LDS update per wavefront
        const uint64_t mv = __ballot(mover);
        uint32_t ls = lifts, dm = dist;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            ls += (uint32_t)__shfl_xor((int)ls, o, 64);
            dm = max(dm, (uint32_t)__shfl_xor((int)dm, o, 64));
        }
        const uint64_t stay = __ballot(live && !mover);
        if (lane == 0) {
            atomicAdd(&s_acc[0], (unsigned long long)__popcll(mv));
            atomicAdd(&s_acc[1], (unsigned long long)ls);
            atomicMax(&s_acc[2], (unsigned long long)dm);
            atomicAdd(&s_acc[3], (unsigned long long)__popcll(stay));
        }
        if (mover) atomicAdd(&s_acc[3 + min(lifts, (uint32_t)PIC_STATS_LEVELS - 1u)], 1ull);
    }
    if (bad) atomicOr(t.status, bad);
    __syncthreads();
    // record layout (pic_rebin_stats): particles, movers, lifts, max_tunnel, lift_hist[]
    for (int i = tid; i < 3 + PIC_STATS_LEVELS; i += blockDim.x) {
        const unsigned long long v = s_acc[i];
        if (i == 2) atomicMax(&out[3], v);
        else if (i < 2) { if (v) atomicAdd(&out[1 + i], v); }
        else if (v) atomicAdd(&out[4 + (i - 3)], v);
    }
    if (blockIdx.x == 0 && tid == 0) atomicAdd(&out[0], (unsigned long long)n);
}

hipError_t launch_rebin_stats(const pic_tree *t, int scheme, const int64_t *old_start, const uint32_t *bins,
                              int shift, int64_t n, void *stats, hipStream_t s) {
    if (n == 0 || !stats) return hipSuccess;
    const int64_t n_bins = n_bins_of(t, scheme);
    const dim3 g(grid_for(n, 256, 2048)), b(256);
    unsigned long long *o = (unsigned long long *)stats;
    if (t->dim == 2) {
        if (scheme == PIC_PIT) PIC_LAUNCH("rebin_stats", (k_rebin_stats<2, 0>), g, b, 0, s, t->dt, old_start, bins, shift, n, (uint32_t)n_bins, o);
        else PIC_LAUNCH("rebin_stats", (k_rebin_stats<2, 1>), g, b, 0, s, t->dt, old_start, bins, shift, n, (uint32_t)n_bins, o);
    } else {
        if (scheme == PIC_PIT) PIC_LAUNCH("rebin_stats", (k_rebin_stats<3, 0>), g, b, 0, s, t->dt, old_start, bins, shift, n, (uint32_t)n_bins, o);
        else PIC_LAUNCH("rebin_stats", (k_rebin_stats<3, 1>), g, b, 0, s, t->dt, old_start, bins, shift, n, (uint32_t)n_bins, o);
    }
    return hipGetLastError();
}

}  // namespace pic
