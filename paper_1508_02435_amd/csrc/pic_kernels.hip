// pic_kernels.hip -- gfx950 kernels of the spacetree PIC hot path (FP64 form).
//
// gather_push  one thread per particle: locate the leaf holding x (arithmetic
//              for uniform subtrees, a short descent otherwise, its top levels
//              in LDS), d-linear gather of E from the 2^d leaf corners, leapfrog
//              kick and drift, periodic wrap, and the new bin of the particle
//              (PIT leaf rank or PIDT dual-cell rank).  SoA streams, coalesced.
// rebin        a stable counting sort by bin that moves every particle record
//              exactly once: (1) per tile of 4096 particles an LDS radix sort
//              of the tile's bins with a stayer/arrival flag, emitting runs;
//              (2) one decoupled-lookback scan over all (bin, flag) keys; (3)
//              per-key run lists give each run its place among the runs of the
//              same key in tile order; (4) an LDS-staged scatter writes each
//              run contiguously.  Atomics touch integer counters only, and
//              every output position is independent of scheduling.
// deposit      a wavefront per bin reduces its particles' weights per corner
//              (PIT) or per 3^d stencil slot (PIDT) in a fixed order; a second
//              pass sums, per vertex, the slots that touch it in a fixed order.
//              No floating-point atomics.
#include <hip/hip_runtime.h>

#include "pic_host.h"

namespace pic {

// ------------------------------------------------------------------ helpers

__constant__ DivMagic c_magic[PIC_MAX_LEVEL + 2] = {
    make_magic(0),  make_magic(1),  make_magic(2),  make_magic(3),  make_magic(4),
    make_magic(5),  make_magic(6),  make_magic(7),  make_magic(8),  make_magic(9),
    make_magic(10), make_magic(11), make_magic(12), make_magic(13), make_magic(14),
    make_magic(15), make_magic(16), make_magic(17), make_magic(18), make_magic(19)};

__device__ __forceinline__ uint32_t div_pow3(uint32_t n, int e) {
    DivMagic m = c_magic[e];
    return (uint32_t)(((uint64_t)n * m.mul) >> m.shift);
}

__device__ __forceinline__ void flag_status(uint32_t *status, uint32_t bit) {
    atomicOr(status, bit);
}

// Load base[idx] with a 32-bit element offset from a wavefront-uniform base
// (a scalar base plus a 32-bit vector offset, no 64-bit address arithmetic).
// Offsets stay below 2^32 bytes for every table and field array (the tree
// builder caps vertex and leaf counts).
template <typename T>
__device__ __forceinline__ T ld_off(const T *base, uint32_t idx) {
    return *(const T *)((const char *)base + idx * (uint32_t)sizeof(T));
}

// Load through the constant address space: with a wavefront-uniform address
// it becomes a scalar load, which takes no vector memory instruction.  Only
// for data no kernel of the launch writes.
__device__ __forceinline__ double ld_const(const double *p, uint32_t idx) {
    return ((const __attribute__((address_space(4))) double *)p)[idx];
}
__device__ __forceinline__ int64_t ld_const(const int64_t *p, uint32_t idx) {
    return ((const __attribute__((address_space(4))) int64_t *)p)[idx];
}
__device__ __forceinline__ uint32_t ld_const(const uint32_t *p, uint32_t idx) {
    return ((const __attribute__((address_space(4))) uint32_t *)p)[idx];
}

__device__ __forceinline__ double x_scaled(double x, double Sd) { return __dmul_rn(x, Sd); }

// Scaled coordinate of one axis.  y = fl(x * S) is the only rounding on the
// way to the cell; T = floor(2y) resolves half cells (dual-cell faces).  The
// clamp keeps indices in range for malformed input (which is flagged).
struct Axis {
    double y;
    uint32_t T;  // floor(2y) in [0, 2S-1]
};

__device__ __forceinline__ Axis scale_axis(double x, double Sd, int S, uint32_t &bad) {
    if (!(x >= 0.0 && x < 1.0)) bad |= (x == x && fabs(x) != __builtin_inf()) ? PIC_DEV_RANGE : PIC_DEV_NONFINITE;
    Axis a;
    a.y = x * Sd;
    double t = floor(2.0 * a.y);
    t = fmin(fmax(t, 0.0), (double)(2 * S - 1));  // fmax drops NaN
    a.T = (uint32_t)t;
    return a;
}

// The same for a position just wrapped into [0,1): fl(x S) < S there, so
// T = floor(2y) <= 2S-1 without a clamp.  A NaN (from a non-finite velocity
// or field) converts to cell 0 and is flagged.
__device__ __forceinline__ Axis scale_wrapped(double x, double Sd, uint32_t &bad) {
    if (x != x) bad |= PIC_DEV_NONFINITE;
    Axis a;
    a.y = __dmul_rn(x, Sd);
    a.T = (uint32_t)floor(__dadd_rn(a.y, a.y));
    return a;
}

// Peano rank of finest cell c of a regular instance: table lookup when the
// level has a table (always, with TAB), else digit by digit.
template <int D, bool TAB>
__device__ __forceinline__ uint32_t regular_rank(const DevTree &t, const DevInst &in, const uint32_t *c) {
    if (TAB || in.ptab >= 0) {
        const uint32_t S = (uint32_t)in.S;
        uint32_t idx = c[0] + __umul24(c[1], S);
        if (D == 3) idx += __umul24(c[D - 1], __umul24(S, S));
        return ld_off(t.peano_tab, (uint32_t)in.ptab + idx);
    }
    return peano_low<D>(c, in.L);
}

// Descent from the root to the leaf holding finest cell I.  Returns the
// forest-wide leaf rank and the leaf's level.  `lds` holds the first
// `lds_n` entries of node_child (the top levels of a single tree).
template <int D>
__device__ __forceinline__ uint32_t descend(const DevTree &t, const DevInst &in, const uint32_t *I,
                                            const int32_t *lds, int lds_n, int &level) {
    int32_t node = in.node_root;
    int lvl = 0;
    int32_t c;
    for (;;) {
        c = (node < lds_n) ? lds[node] : t.node_child[node];
        if (c < 0) break;
        const int e = in.L - lvl - 1;
        uint32_t slot = 0, m = 1;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            uint32_t q = div_pow3(I[k], e);
            slot += (q - 3u * (q / 3u)) * m;
            m *= 3u;
        }
        node = c + (int32_t)slot;
        ++lvl;
    }
    const uint32_t u = (uint32_t)(-c - 1);
    const uint32_t meta = t.uni_meta[u];
    const int depth = (int)(meta >> 8);
    level = lvl + depth;
    uint32_t a[D];
#pragma unroll
    for (int k = 0; k < D; ++k) a[k] = div_pow3(I[k], in.L - level);
    return t.uni_base[u] + peano_low<D>(a, depth);
}

// Instance of particle p in a forest (binary search over particle offsets).
// The lanes of a wavefront hold consecutive slots, mostly of one instance:
// the first active lane's instance is found with scalar loads, and only
// lanes outside it search on their own.
__device__ __forceinline__ int inst_of(const int64_t *start, int n_inst, int64_t p) {
    const int l = __builtin_ctzll(__ballot(1));
    const uint64_t pu = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)p, l)) |
                        ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)p >> 32), l) << 32);
    int lo = 0, hi = n_inst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (ld_const(start, (uint32_t)mid) <= (int64_t)pu) lo = mid; else hi = mid - 1;
    }
    if (ld_const(start, (uint32_t)lo) <= p && p < ld_const(start, (uint32_t)lo + 1u)) return lo;
    lo = 0;
    hi = n_inst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= p) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// New bin of a particle from its scaled axes.
template <int D, int SCHEME, bool REG>
__device__ __forceinline__ uint32_t bin_of(const DevTree &t, const DevInst &in, const Axis *ax,
                                           const int32_t *lds, int lds_n) {
    if (REG) {
        uint32_t c[D];
        if (SCHEME == PIC_PIT) {
#pragma unroll
            for (int k = 0; k < D; ++k) c[k] = ax[k].T >> 1;
            return (uint32_t)in.leaf_off + regular_rank<D, true>(t, in, c);
        } else {
            const uint32_t S = (uint32_t)in.S, half = (S - 1u) >> 1;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                uint32_t J = (ax[k].T + 1u) >> 1;       // nearest finest vertex, ties up
                if (J >= S) J -= S;
                J += half;                              // shifted lattice of nested dual cells
                if (J >= S) J -= S;
                c[k] = J;
            }
            return (uint32_t)in.pidt_off + regular_rank<D, true>(t, in, c);
        }
    } else {
        uint32_t I[D];
#pragma unroll
        for (int k = 0; k < D; ++k) I[k] = ax[k].T >> 1;
        int lev;
        const uint32_t rank = descend<D>(t, in, I, lds, lds_n, lev);
        if (SCHEME == PIC_PIT) return rank;
        const int e = in.L - lev;
        const uint32_t s = pow3_u32(e);
        int corner = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const uint32_t a = div_pow3(I[k], e);
            if (ax[k].T >= (2u * a + 1u) * s) corner |= 1 << k;
        }
        return (uint32_t)t.leaf_pidt[(int64_t)rank * (1 << D) + corner];
    }
}

template <bool REG>
__device__ __forceinline__ int stage_nodes(const DevTree &t, const DevInst &in, int32_t *lds) {
    if (REG) return 0;
    const int n = in.lds_nodes;
    for (int i = threadIdx.x; i < n; i += blockDim.x) lds[i] = t.node_child[in.node_root + i];
    __syncthreads();
    return in.node_root + n;  // descent indices are forest-wide; entries below this come from LDS
}

struct F64Ptrs {
    double *x[3];
    double *v[3];
    const double *E[3];
    double *Ep[3];
};

// ------------------------------------------------------------ gather + push
//
// Arithmetic contract (matches a serial IEEE evaluation, no FMA contraction):
//   f_k = (y_k - a_k s) * fl(1/s),  g_k = 1 - f_k,
//   w_c = prod_k (bit k of c ? f_k : g_k)  multiplied in axis order,
//   E_j = w_0 E_j[v_0] + w_1 E_j[v_1] + ...  in corner order,
//   v_j = v_j + qmdt E_j,  x_j = x_j + v_j dt,  x_j = x_j - floor(x_j), 1 -> 0.
// push_one updates xv, vv in place, stores E_p when P.Ep[0] is set, and
// returns the particle's new bin (0 without KEY); non-finite or out-of-box
// input sets bits in `bad`.
template <int D, int SCHEME, bool REG, bool EP = true, bool KEY = true>
__device__ __forceinline__ uint32_t push_one(const DevTree &t, const DevInst &in, const F64Ptrs &P,
                                             const int32_t *lds, int lds_n, double (&xv)[D], double (&vv)[D],
                                             double qmdt, double dt, int64_t p, uint32_t &bad) {
    Axis ax[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        ax[k] = scale_axis(xv[k], in.Sd, in.S, bad);
        if (!(vv[k] - vv[k] == 0.0)) bad |= PIC_DEV_NONFINITE;
    }
    // leaf holding x: corner vertex ids and the local coordinates f, g
    uint32_t I[D];
#pragma unroll
    for (int k = 0; k < D; ++k) I[k] = ax[k].T >> 1;
    uint32_t vid[1 << D];
    double f[D], g[D];
    if (REG) {
        // finest cell I: corner c is I + bits of c per axis, periodic, so the
        // ids follow from the id of corner 0 by per-axis steps
        const uint32_t S = (uint32_t)in.S;
        uint32_t stride = 1, v0 = (uint32_t)in.vtx_off;
        uint32_t step[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            v0 += __umul24(I[k], stride);
            step[k] = I[k] + 1u == S ? stride - __umul24(S, stride) : stride;   // wraps modulo 2^32
            stride = __umul24(stride, S);
        }
#pragma unroll
        for (int c = 0; c < (1 << D); ++c) {
            uint32_t v = v0;
#pragma unroll
            for (int k = 0; k < D; ++k)
                if ((c >> k) & 1) v += step[k];
            vid[c] = v;
        }
        // s = 1 and fl(1/s) = 1: f = y - I exactly as (y - I s) * fl(1/s)
#pragma unroll
        for (int k = 0; k < D; ++k) {
            f[k] = __dsub_rn(ax[k].y, (double)I[k]);
            g[k] = __dsub_rn(1.0, f[k]);
        }
    } else {
        int lev;
        const uint32_t rank = descend<D>(t, in, I, lds, lds_n, lev);
#pragma unroll
        for (int c = 0; c < (1 << D); ++c) vid[c] = (uint32_t)t.leaf_vtx[(int64_t)rank * (1 << D) + c];
        const uint32_t su = pow3_u32(in.L - lev);
        const double s = (double)su;
        const double rinv = in.rinv[lev];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const uint32_t a = div_pow3(I[k], in.L - lev);
            f[k] = __dmul_rn(__dsub_rn(ax[k].y, (double)a * s), rinv);
            g[k] = __dsub_rn(1.0, f[k]);
        }
    }
    double w[1 << D];
#pragma unroll
    for (int c = 0; c < (1 << D); ++c) {
        double wc = (c & 1) ? f[0] : g[0];
#pragma unroll
        for (int k = 1; k < D; ++k) wc = __dmul_rn(wc, ((c >> k) & 1) ? f[k] : g[k]);
        w[c] = wc;
    }
    // Field at the corners.  Particles are stored by bin, so the lanes of a
    // wavefront mostly share one or two cells: up to two passes serve the
    // lanes whose cell is that of the first pending lane (the id of corner 0
    // names the cell) with scalar loads, and only the lanes left gather per
    // lane.  The values, and so the arithmetic, are the same either way.
    double Ec[D == 2 ? 4 : 1][D];   // 2D: the corner values; 3D: the interpolant ef instead
    double ef[D];
    uint64_t pend = __ballot(1);
    const uint32_t lane = __lane_id();
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        if (!pend) break;
        const int l = __builtin_ctzll(pend);
        const uint32_t v0u = (uint32_t)__builtin_amdgcn_readlane((int)vid[0], l);
        const bool mine = vid[0] == v0u;
        pend &= ~__ballot(mine);
        uint32_t vu[1 << D];
#pragma unroll
        for (int c = 0; c < (1 << D); ++c) vu[c] = (uint32_t)__builtin_amdgcn_readlane((int)vid[c], l);
        if constexpr (D == 2) {
#pragma unroll
            for (int c = 0; c < (1 << D); ++c)
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    const double eu = ld_const(P.E[j], vu[c]);
                    if (mine) Ec[c][j] = eu;
                }
        } else {
            // 3D: the 24 corner values stay in scalar registers; every lane
            // forms this cell's interpolant (same operation order) and the
            // lanes of the cell keep it, so no vector registers hold them
#pragma unroll
            for (int j = 0; j < D; ++j) {
                double e = __dmul_rn(w[0], ld_const(P.E[j], vu[0]));
#pragma unroll
                for (int c = 1; c < (1 << D); ++c) e = __dadd_rn(e, __dmul_rn(w[c], ld_const(P.E[j], vu[c])));
                if (mine) ef[j] = e;
            }
        }
    }
    if ((pend >> lane) & 1ull) {
        if constexpr (D == 2) {
#pragma unroll
            for (int c = 0; c < (1 << D); ++c)
#pragma unroll
                for (int j = 0; j < D; ++j) Ec[c][j] = ld_off(P.E[j], vid[c]);
        } else {
#pragma unroll
            for (int j = 0; j < D; ++j) {
                double e = __dmul_rn(w[0], ld_off(P.E[j], vid[0]));
#pragma unroll
                for (int c = 1; c < (1 << D); ++c) e = __dadd_rn(e, __dmul_rn(w[c], ld_off(P.E[j], vid[c])));
                ef[j] = e;
            }
        }
    }
#pragma unroll
    for (int j = 0; j < D; ++j) {
        double e;
        if constexpr (D == 2) {
            e = __dmul_rn(w[0], Ec[0][j]);
#pragma unroll
            for (int c = 1; c < (1 << D); ++c) e = __dadd_rn(e, __dmul_rn(w[c], Ec[c][j]));
        } else {
            e = ef[j];
        }
        if (EP && P.Ep[0]) P.Ep[j][p] = e;
        double vj = __dadd_rn(vv[j], __dmul_rn(qmdt, e));
        double xj = __dadd_rn(xv[j], __dmul_rn(vj, dt));
        xj = __dsub_rn(xj, floor(xj));
        if (xj == 1.0) xj = 0.0;
        vv[j] = vj;
        xv[j] = xj;
    }
    if (!KEY) return 0u;
#pragma unroll
    for (int k = 0; k < D; ++k) ax[k] = scale_wrapped(xv[k], in.Sd, bad);
    return bin_of<D, SCHEME, REG>(t, in, ax, lds, lds_n);
}

template <int D, int SCHEME, bool REG, bool MULTI>
__global__ __launch_bounds__(256) void k_gather_push(DevTree t, DevInst in0, F64Ptrs P, int64_t n,
                                                     double qmdt0, double dt0, const double *qmdt_arr,
                                                     const double *dt_arr, const int64_t *inst_start,
                                                     uint32_t *bin_out) {
    __shared__ int32_t lds[REG ? 1 : PIC_LDS_NODES];
    const int lds_n = MULTI ? 0 : stage_nodes<REG>(t, in0, lds);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        int ii = 0;
        if (MULTI) ii = inst_of(inst_start, t.n_inst, p);
        const DevInst &in = MULTI ? t.inst[ii] : in0;
        const double qmdt = (MULTI && qmdt_arr) ? qmdt_arr[ii] : qmdt0;
        const double dt = (MULTI && dt_arr) ? dt_arr[ii] : dt0;
        uint32_t bad = 0;
        double xv[D], vv[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            xv[k] = P.x[k][p];
            vv[k] = P.v[k][p];
        }
        const uint32_t nb = push_one<D, SCHEME, REG>(t, in, P, lds, lds_n, xv, vv, qmdt, dt, p, bad);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            P.x[k][p] = xv[k];
            P.v[k][p] = vv[k];
        }
        bin_out[p] = nb;
        if (bad) flag_status(t.status, bad);
    }
}

template <int D, int SCHEME, bool REG, bool MULTI>
__global__ __launch_bounds__(256) void k_locate(DevTree t, DevInst in0, F64Ptrs P, int64_t n,
                                                const int64_t *inst_start, uint32_t *bin_out) {
    __shared__ int32_t lds[REG ? 1 : PIC_LDS_NODES];
    const int lds_n = MULTI ? 0 : stage_nodes<REG>(t, in0, lds);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        const DevInst &in = MULTI ? t.inst[inst_of(inst_start, t.n_inst, p)] : in0;
        uint32_t bad = 0;
        Axis ax[D];
#pragma unroll
        for (int k = 0; k < D; ++k) ax[k] = scale_axis(P.x[k][p], in.Sd, in.S, bad);
        bin_out[p] = bin_of<D, SCHEME, REG>(t, in, ax, lds, lds_n);
        if (bad) flag_status(t.status, bad);
    }
}

// ------------------------------------------------------------- block scans

// Exclusive scan of one uint32 per thread over a 256-thread block; returns the
// exclusive prefix and writes the block total to *total.  `wsum` is 4 words of
// LDS.  Fixed combination order, so the result is deterministic.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *wsum, uint32_t *total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        uint32_t s = wsum[w];
        if (w < wv) base += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return base + x - v;
}

// ------------------------------------------------------------------- rebin

constexpr int RB_THREADS = 256;
constexpr int KLIST_CAP = 128;  // runs per key listed directly by the fused step's ranking
constexpr int RB_MAX_TILE = 4096;

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

struct RebinScratch {
    uint32_t *tile_bin;   // n_tiles * 2: bin holding the first slot, 1 + bin holding the last slot
    uint16_t *perm;       // n_tiles * TILE: tile-local source index per sorted slot
    uint32_t *run_key;    // n_tiles * TILE
    uint32_t *run_info;   // start | count << 16
    uint32_t *run_dest;   // n_tiles * TILE
    uint32_t *tile_nruns; // n_tiles
    uint32_t *key_cnt;    // 2*n_bins (zeroed per call)
    uint32_t *key_nruns;  // 2*n_bins (zeroed per call)
    uint32_t *key_fill;   // 2*n_bins (zeroed per call)
    uint64_t *key_cn;     // 2*n_bins (zeroed per call): fused step, count << 32 | runs per key
    uint32_t *key_base;   // 2*n_bins
    uint32_t *list_off;   // 2*n_bins + 1
    uint32_t *list;       // total runs <= n_tiles * TILE
    uint64_t *scan_state; // per scan block (zeroed per call)
    uint32_t *scan_ctr;   // dynamic block counter (zeroed per call)
    uint64_t *run_wcnt;   // n_tiles * TILE: fused step, 16-bit count per wavefront
    uint32_t *meta;       // n_tiles * TILE: fused step, run index | rank << 16 per particle
    uint32_t *keys;       // n_tiles * TILE: fused step (three-pass form), key per particle
    uint32_t *klist;      // 2*n_bins * KLIST_CAP: fused step, run addresses per key (arrival order)
    uint32_t *khead;      // 2*n_bins (zeroed per call): runs of a key past KLIST_CAP, a linked list
    uint32_t *knext;      // n_tiles * TILE: next run of that list (run address + 1; 0 ends it)
    uint32_t *wave_bin;   // n_tiles * TILE / 64: old bin of slot 64 c (sorted input), for the FP32 form
};

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
constexpr int SCAN_IPT = 8;
constexpr int SCAN_TILE = 256 * SCAN_IPT;
constexpr uint64_t ST_AGG = 1ull << 62, ST_PRE = 2ull << 62, ST_VAL = (1ull << 62) - 1;

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

// Pass 3b: a run's place among the runs of its key is the particle count of
// the key's runs from earlier tiles (lower run address).  Each wavefront
// takes four keys, one per 16-lane group; a list of up to 16 runs is sorted by
// address with a bitonic sort inside its group and prefix-summed.  Longer
// lists are then handled by the whole wavefront: up to 64 runs with a 64-lane
// bitonic sort, beyond that by counting the smaller addresses per run.
template <int W>
__device__ __forceinline__ void place_sorted(const RebinScratch &sc, const uint32_t *lst, uint32_t l0, uint32_t len,
                                             uint32_t kb, int sub) {
    uint32_t a = 0xffffffffu, c = 0;
    if ((uint32_t)sub < len) {
        a = lst[l0 + sub];
        c = sc.run_info[a] >> 16;
    }
#pragma unroll
    for (int k = 2; k <= W; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint32_t oa = (uint32_t)__shfl_xor((int)a, j, 64);
            const uint32_t oc = (uint32_t)__shfl_xor((int)c, j, 64);
            const bool up = (sub & k) == 0;
            const bool lower = (sub & j) == 0;
            const bool take = lower == up ? (oa < a) : (oa > a);
            if (take) { a = oa; c = oc; }
        }
    }
    uint32_t x = c;
#pragma unroll
    for (int o = 1; o < W; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, o, W);
        if (sub >= o) x += y;
    }
    if ((uint32_t)sub < len) sc.run_dest[a] = kb + x - c;
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

// Fused step, middle.  Scan: each block of SP_THREADS threads scans the
// (count, runs) pairs of SP_KEYS keys; its first wavefront publishes the
// block's aggregate and looks back over up to 64 predecessors at a time (one
// lane per predecessor) for the exclusive prefix.  Place: per key, its runs
// (the direct list the ranking filled, then for keys with more than KLIST_CAP
// runs the linked rest) sorted by run address, i.e. tile order, and given
// their destinations.
constexpr int SP_THREADS = 256;
constexpr int SP_KPT = 16;                      // keys per thread
constexpr int SP_KEYS = SP_THREADS * SP_KPT;

__global__ __launch_bounds__(SP_THREADS) void k_step_scan(uint32_t n_keys, uint32_t n_bins, int64_t n, RebinScratch sc,
                                                          int64_t *new_start, uint32_t *status) {
    // Blocks are dispatched in index order, so every predecessor a block
    // waits for is already running (the wait is bounded all the same).
    __shared__ uint32_t s_wsum[4];
    __shared__ uint64_t s_excl;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const uint32_t bid = blockIdx.x;
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
                                              uint32_t kb, int lane) {
    uint32_t a0 = ~0u, c0 = 0u, a1 = ~0u, c1 = 0u;
    if ((uint32_t)lane < len) {
        a0 = lst[l0 + lane];
        c0 = sc.run_info[a0] >> 16;
    }
    if ((uint32_t)lane + 64u < len) {
        a1 = lst[l0 + 64 + lane];
        c1 = sc.run_info[a1] >> 16;
    }
    uint32_t b0 = 0u, b1 = 0u;
    for (int j = 0; j < 64; ++j) {
        const uint32_t x0 = (uint32_t)__builtin_amdgcn_readlane((int)a0, j);
        const uint32_t y0 = (uint32_t)__builtin_amdgcn_readlane((int)c0, j);
        const uint32_t x1 = (uint32_t)__builtin_amdgcn_readlane((int)a1, j);
        const uint32_t y1 = (uint32_t)__builtin_amdgcn_readlane((int)c1, j);
        b0 += (x0 < a0 ? y0 : 0u) + (x1 < a0 ? y1 : 0u);
        b1 += (x0 < a1 ? y0 : 0u) + (x1 < a1 ? y1 : 0u);
    }
    if ((uint32_t)lane < len) sc.run_dest[a0] = kb + b0;
    if ((uint32_t)lane + 64u < len) sc.run_dest[a1] = kb + b1;
}

__global__ __launch_bounds__(256) void k_step_place(RebinScratch sc, uint32_t n_keys) {
    const int lane = threadIdx.x & 63;
    const int grp = lane >> 4, sub = lane & 15;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t k0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * 4; k0 < n_keys;
         k0 += waves * 4) {
        const int64_t key = k0 + grp;
        uint32_t len = 0, kb = 0;
        if (key < n_keys) {
            len = (uint32_t)sc.key_cn[key];
            kb = sc.key_base[key];
        }
        if (__ballot(len != 0u) == 0) continue;   // four empty keys
        if (len <= 16) place_sorted<16>(sc, sc.klist, (uint32_t)(key * KLIST_CAP), len, kb, sub);
        for (int g = 0; g < 4; ++g) {
            const int64_t gk = k0 + g;
            const uint32_t glen = (uint32_t)__shfl((int)len, g * 16, 64);
            const uint32_t gkb = (uint32_t)__shfl((int)kb, g * 16, 64);
            if (glen <= 16) continue;
            if (glen <= 64u) {
                place_sorted<64>(sc, sc.klist, (uint32_t)(gk * KLIST_CAP), glen, gkb, lane);
                continue;
            }
            if (glen <= (uint32_t)KLIST_CAP) {
                place_counted(sc, sc.klist, (uint32_t)(gk * KLIST_CAP), glen, gkb, lane);
                continue;
            }
            // a long list: gathered into its exact slot range of the list
            // array (direct part by the lanes, linked part by lane 0), then
            // every run counts the runs before it
            const uint32_t l0 = sc.list_off[gk];
            for (int i = lane; i < KLIST_CAP; i += 64) sc.list[l0 + i] = sc.klist[gk * KLIST_CAP + i];
            if (lane == 0) {
                uint32_t q = KLIST_CAP;
                for (uint32_t e = sc.khead[gk]; e != 0u && q < glen; e = sc.knext[e - 1u]) sc.list[l0 + q++] = e - 1u;
            }
            __threadfence();   // lane 0's entries visible to the other lanes' loads
            for (uint32_t q = lane; q < glen; q += 64) {
                const uint32_t a = sc.list[l0 + q];
                uint32_t before = 0;
                for (uint32_t j = l0; j < l0 + glen; ++j) {
                    const uint32_t bb = sc.list[j];
                    if (bb < a) before += sc.run_info[bb] >> 16;
                }
                sc.run_dest[a] = gkb + before;
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

// ------------------------------------------------------------- fused step
//
// A whole step in two passes over the particles.  Both passes push the same
// tile of particles with the same arithmetic, so they agree on every new bin
// without the bins ever going through memory.
//   count: per tile, the number of particles of each key 2*bin + arrived,
//          split by wavefront (wavefront w owns the tile's slots
//          [w*64*IPT, (w+1)*64*IPT), in order).  These become the tile's runs.
//   move:  the runs' destinations are known (scan + placement); each
//          particle is written to its run's destination plus its rank among
//          the earlier particles of the tile with the same key.
// A particle stays iff its slot lies in its new bin's old segment.
//
// Keys are gathered per tile in an LDS open-addressing table of 2*TILE
// slots, so insertion always finds a free slot; every lane inserts and counts
// its own key (integer atomics, so the counts do not depend on timing).

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

constexpr int STEP_RCAP = 256;

template <int IPT>
struct StepShape {
    static constexpr int TILE = RB_THREADS * IPT;
    static constexpr int HB = IPT == 4 ? 11 : (IPT == 8 ? 12 : 13);   // 2*TILE table slots
    static constexpr int H = 1 << HB;
    static_assert(H == 2 * TILE, "table size");
};

// Loads and pushes the tile's particles (slot w*64*IPT + j*64 + lane of
// thread (w, lane)) and forms their keys; ~0 marks slots past the end.
template <int D, int SCHEME, bool REG, bool MULTI, int IPT>
__device__ __forceinline__ void step_push_tile(const DevTree &t, const DevInst &in0, const F64Ptrs &P, int64_t n,
                                               int64_t lo, double qmdt0, double dt0, const double *qa,
                                               const double *da, const int64_t *inst_start,
                                               const int64_t *old_start, uint32_t n_bins, const int32_t *lds,
                                               int lds_n, double (&xv)[IPT][D], double (&vv)[IPT][D],
                                               uint32_t (&key)[IPT], uint32_t &bad) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t base = lo + (int64_t)w * 64 * IPT + lane;
    uint32_t nb[IPT];
    if (!MULTI && lo + RB_THREADS * IPT <= n) {
        // full tile: no per-slot guards, so the rounds form straight-line code
        // and their loads (state, field, offsets) overlap
#pragma unroll
        for (int j = 0; j < IPT; ++j)
#pragma unroll
            for (int k = 0; k < D; ++k) {
                xv[j][k] = P.x[k][base + 64 * j];
                vv[j][k] = P.v[k][base + 64 * j];
            }
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            uint32_t b = push_one<D, SCHEME, REG, false>(t, in0, P, lds, lds_n, xv[j], vv[j], qmdt0, dt0,
                                                         base + 64 * j, bad);
            if (b >= n_bins) bad |= PIC_DEV_RANGE;
            nb[j] = min(b, n_bins - 1);
        }
    } else {
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const int64_t p = base + 64 * j;
#pragma unroll
            for (int k = 0; k < D; ++k) {
                xv[j][k] = p < n ? P.x[k][p] : 0.0;
                vv[j][k] = p < n ? P.v[k][p] : 0.0;
            }
        }
#pragma unroll
        for (int j = 0; j < IPT; ++j) {
            const int64_t p = base + 64 * j;
            nb[j] = ~0u;
            if (p < n) {
                int ii = 0;
                if (MULTI) ii = inst_of(inst_start, t.n_inst, p);
                const DevInst &in = MULTI ? t.inst[ii] : in0;
                const double qmdt = (MULTI && qa) ? qa[ii] : qmdt0;
                const double dt = (MULTI && da) ? da[ii] : dt0;
                uint32_t b = push_one<D, SCHEME, REG, false>(t, in, P, lds, lds_n, xv[j], vv[j], qmdt, dt, p, bad);
                if (b >= n_bins) bad |= PIC_DEV_RANGE;
                nb[j] = min(b, n_bins - 1);
            }
        }
    }
    // stayer iff the slot lies in its new bin's old segment
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const int64_t p = base + 64 * j;
        key[j] = ~0u;
        if (nb[j] != ~0u) {
            bool stay = false;
            if (old_start) {
                const int64_t s0 = old_start[nb[j]], s1 = old_start[nb[j] + 1];
                stay = s0 <= p && p < s1;
            }
            key[j] = 2u * nb[j] + (stay ? 0u : 1u);
        }
    }
}

template <int D, int SCHEME, bool REG, bool MULTI, int IPT>
__global__ __launch_bounds__(RB_THREADS) void k_step_count(DevTree t, DevInst in0, F64Ptrs P, int64_t n,
                                                          double qmdt0, double dt0, const double *qa,
                                                          const double *da, const int64_t *inst_start,
                                                          const int64_t *old_start, uint32_t n_bins,
                                                          RebinScratch sc) {
    using SS = StepShape<IPT>;
    __shared__ uint32_t s_key[SS::H];
    __shared__ uint64_t s_cnt[SS::H];   // 16-bit count per wavefront
    __shared__ uint32_t s_nruns;
    __shared__ int32_t lds[REG ? 1 : PIC_LDS_NODES];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t tile = blockIdx.x;
    const int64_t lo = tile * SS::TILE;
    for (int i = tid; i < SS::H; i += RB_THREADS) {
        s_key[i] = 0u;
        s_cnt[i] = 0u;
    }
    if (tid == 0) s_nruns = 0u;
    const int lds_n = MULTI ? 0 : stage_nodes<REG>(t, in0, lds);
    double xv[IPT][D], vv[IPT][D];
    uint32_t key[IPT];
    uint32_t bad = 0;
    step_push_tile<D, SCHEME, REG, MULTI, IPT>(t, in0, P, n, lo, qmdt0, dt0, qa, da, inst_start, old_start, n_bins,
                                               lds, lds_n, xv, vv, key, bad);
    if (bad) flag_status(t.status, bad);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        if (key[j] == ~0u) continue;
        uint32_t slot = table_find<SS::HB>(s_key, key[j]);         // most keys are in already
        if (slot == ~0u) slot = table_insert<SS::HB>(s_key, key[j]);
        atomicAdd((unsigned long long *)&s_cnt[slot], 1ull << (16 * w));
    }
    __syncthreads();
    for (int i = tid; i < SS::H; i += RB_THREADS) {
        const uint32_t k1 = s_key[i];
        if (!k1) continue;
        const uint64_t c = s_cnt[i];
        const uint32_t tot = (uint32_t)((c & 0xffffu) + ((c >> 16) & 0xffffu) + ((c >> 32) & 0xffffu) + (c >> 48));
        const uint32_t ri = atomicAdd(&s_nruns, 1u);
        sc.run_key[lo + ri] = k1 - 1u;
        sc.run_info[lo + ri] = tot << 16;
        sc.run_wcnt[lo + ri] = c;
        atomicAdd(&sc.key_cnt[k1 - 1u], tot);
        atomicAdd(&sc.key_nruns[k1 - 1u], 1u);
    }
    __syncthreads();
    if (tid == 0) sc.tile_nruns[tile] = s_nruns;
}

// Move pass.  Each slot is ranked within its run in tile order (wavefront
// chunks in order, lanes in order) and written to the run's destination plus
// that rank.  The tile's run table is loaded together with the particles
// (its first RB_THREADS entries speculatively: the tile's run area always
// holds them), so the block waits for memory once and passes one barrier.
template <int D, int SCHEME, bool REG, bool MULTI, int IPT>
__global__ __launch_bounds__(RB_THREADS) void k_step_move(DevTree t, DevInst in0, F64Ptrs P, int64_t n,
                                                         double qmdt0, double dt0, const double *qa,
                                                         const double *da, const int64_t *inst_start,
                                                         const int64_t *old_start, uint32_t n_bins,
                                                         RebinScratch sc, F64Ptrs out, Cols extra) {
    using SS = StepShape<IPT>;
    constexpr int TILE = SS::TILE;
    __shared__ uint32_t s_key[SS::H];
    __shared__ uint16_t s_run[SS::H];
    __shared__ uint32_t s_cur[4][TILE];   // per wavefront: next destination of each run
    __shared__ unsigned long long s_msk[4][STEP_RCAP];
    __shared__ int32_t lds[REG ? 1 : PIC_LDS_NODES];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t tile = blockIdx.x;
    const int64_t lo = tile * TILE;
    for (int i = tid; i < SS::H; i += RB_THREADS) s_key[i] = 0u;
    for (int i = tid; i < 4 * STEP_RCAP; i += RB_THREADS) (&s_msk[0][0])[i] = 0ull;
    const uint32_t nr = min(sc.tile_nruns[tile], (uint32_t)TILE);
    const uint32_t rk0 = sc.run_key[lo + tid];
    const uint64_t rw0 = sc.run_wcnt[lo + tid];
    const uint32_t rd0 = sc.run_dest[lo + tid];
    const int lds_n = MULTI ? 0 : stage_nodes<REG>(t, in0, lds);
    double xv[IPT][D], vv[IPT][D];
    uint32_t key[IPT];
    uint32_t bad = 0;
    step_push_tile<D, SCHEME, REG, MULTI, IPT>(t, in0, P, n, lo, qmdt0, dt0, qa, da, inst_start, old_start, n_bins,
                                               lds, lds_n, xv, vv, key, bad);
    __syncthreads();                          // table cleared (all waves past the clear)
    for (uint32_t q = tid; q < nr; q += RB_THREADS) {
        const bool first = q < (uint32_t)RB_THREADS;
        const uint32_t k = first ? rk0 : sc.run_key[lo + q];
        const uint64_t c = first ? rw0 : sc.run_wcnt[lo + q];
        uint32_t d = first ? rd0 : sc.run_dest[lo + q];
        const uint32_t slot = table_insert<SS::HB>(s_key, k);
        s_run[slot] = (uint16_t)q;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            s_cur[v][q] = d;
            d += (uint32_t)((c >> (16 * v)) & 0xffffu);
        }
    }
    __syncthreads();
    // rank: the lanes of a round that share a run OR their bit into the run's
    // mask, read it back, and the lowest of them advances the run's cursor;
    // runs numbered STEP_RCAP and above go through a ballot loop
    uint32_t dst[IPT];
    uint32_t miss = 0;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        const bool valid = key[j] != ~0u;
        dst[j] = ~0u;
        uint32_t ri = ~0u;
        if (valid) {
            const uint32_t slot = table_find<SS::HB>(s_key, key[j]);
            if (slot != ~0u) ri = s_run[slot];
            else miss = 1;
        }
        const bool fast = ri < (uint32_t)STEP_RCAP;
        if (fast) atomicOr(&s_msk[w][ri], 1ull << lane);
        uint64_t m = 0;
        uint32_t b = 0;
        if (fast) {
            m = s_msk[w][ri];
            b = s_cur[w][ri];
        }
        const uint32_t below = lanes_below(m);
        if (fast && below == 0) {
            s_cur[w][ri] = b + (uint32_t)__popcll(m);
            s_msk[w][ri] = 0ull;
        }
        if (fast) dst[j] = b + below;
        const bool slow = ri != ~0u && !fast;
        uint64_t todo = __ballot(slow);
        while (todo) {
            const int leader = __builtin_ctzll(todo);
            const uint32_t r = (uint32_t)__shfl((int)ri, leader, 64);
            const uint64_t ms = __ballot(slow && ri == r);
            todo &= ~ms;
            uint32_t bs = 0;
            if (lane == leader) {
                bs = s_cur[w][r];
                s_cur[w][r] = bs + (uint32_t)__popcll(ms);
            }
            bs = (uint32_t)__shfl((int)bs, leader, 64);
            if (slow && ri == r) dst[j] = bs + lanes_below(ms);
        }
        if (dst[j] != ~0u && dst[j] >= (uint32_t)n) {   // inconsistent input: never write out of range
            dst[j] = ~0u;
            miss = 1;
        }
    }
    if (miss) flag_status(t.status, PIC_DEV_RANGE);
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        if (dst[j] == ~0u) continue;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            out.x[k][dst[j]] = xv[j][k];
            out.v[k][dst[j]] = vv[j][k];
        }
    }
    const int64_t base = lo + (int64_t)w * 64 * IPT + lane;
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
}

// ------------------------------------------------------ fused step, ranked
//
// The same two passes, with the ranking moved into the first one.
//   rank:  per tile, each particle's key 2*bin + arrived and its rank among
//          the tile's particles with that key (tile order), stored as one
//          word per particle: run index | rank << 16.  The tile's runs (key,
//          count) go to the run table as before.
//   emit:  push again (no bin), destination = run destination + rank.  No
//          LDS and no barrier for regular trees.
// Both passes push with the same arithmetic, so the emitted state is the
// state the rank pass binned.
//
// Ranking inside a round (64 lanes, one slot each) without ordering
// assumptions on LDS atomics: every lane writes its lane id to a per-wave tag
// of its table slot and reads the tag back, which gives all lanes of a slot
// the same representative lane; each lane then ORs its bit into the mask of
// that representative and reads the mask, whose lanes below its own give its
// rank.  The lowest lane of a mask advances the wave's count of the slot.
// The representative a tag ends up with depends on timing, the masks do not.

template <int IPT>
struct RankShape {
    static constexpr int TILE = RB_THREADS * IPT;
    static constexpr int HB = IPT == 4 ? 10 : (IPT == 8 ? 11 : 12);   // TILE table slots
    static constexpr int H = 1 << HB;
    static_assert(H == TILE, "table size");
};

// Entries at the head of a tile's run table that the emit pass loads with
// the tile's state (most tiles have fewer runs).
constexpr int RUN_HEAD = 256;

// Block b's tile when the tiles are spread over the chip's 8 XCDs in
// contiguous chunks (consecutive blocks go to consecutive XCDs), so that the
// tiles an XCD runs at the same time are neighbours and share its L2.
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t tiles, int on) {
    if (!on) return b;
    const int64_t x = b & 7, k = b >> 3, q = tiles >> 3, r = tiles & 7;
    return x * q + (x < r ? x : r) + k;
}

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
        if (pos[e] < (uint32_t)KLIST_CAP) sc.klist[(int64_t)k * KLIST_CAP + pos[e]] = a;
        else sc.knext[a] = atomicExch(&sc.khead[k], a + 1u);
    }
    __syncthreads();
    if (tid == 0) sc.tile_nruns[tile] = total & 0xffffu;
    const int64_t pbase = lo + (int64_t)w * 64 * IPT + lane;
#pragma unroll
    for (int j = 0; j < IPT; ++j) {
        if (key[j] == ~0u) continue;
        meta[pbase + 64 * j] = S.key[slot[j]] | ((S.wc[w][slot[j]] + rk[j]) << 16);
    }
}

template <int D, int SCHEME, bool REG, bool MULTI, int IPT>
__global__ __launch_bounds__(RB_THREADS) void k_step_rank(DevTree t, DevInst in0, F64Ptrs P, int64_t n,
                                                         double qmdt0, double dt0, const double *qa,
                                                         const double *da, const int64_t *inst_start,
                                                         const int64_t *old_start, uint32_t n_bins,
                                                         RebinScratch sc, uint32_t *meta, int xcd) {
    using RS = RankShape<IPT>;
    __shared__ RankSmem<IPT> S;
    __shared__ int32_t lds[REG ? 1 : PIC_LDS_NODES];
    const int64_t tile = xcd_tile(blockIdx.x, gridDim.x, xcd);
    const int64_t lo = tile * RS::TILE;
    rank_clear<IPT>(S);
    const int lds_n = MULTI ? 0 : stage_nodes<REG>(t, in0, lds);
    double xv[IPT][D], vv[IPT][D];
    uint32_t key[IPT];
    uint32_t bad = 0;
    step_push_tile<D, SCHEME, REG, MULTI, IPT>(t, in0, P, n, lo, qmdt0, dt0, qa, da, inst_start, old_start, n_bins,
                                               lds, lds_n, xv, vv, key, bad);
    if (bad) flag_status(t.status, bad);
    __syncthreads();   // table cleared
    tile_rank<IPT>(S, key, tile, lo, sc, meta);
}

// Key pass of the three-pass form: one particle per thread, pushed, its key
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

// Group pass of the three-pass form: the tile ranking of k_step_rank over
// keys read from memory.
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

// ----------------------------------------------------------------- deposit

// Sum over groups of G consecutive lanes (butterfly inside the group, fixed
// order, so the result is the same on every run).
// A double moved across lanes by a DPP pattern (both halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Sum over groups of G consecutive lanes.  Inside a row of 16 lanes the
// partners come by DPP (swap neighbours, swap pairs, mirror the half row,
// mirror the row), across rows by lane shuffles.  Each step adds a lane's
// value and its partner's, and a + b == b + a, so every lane of a group ends
// with the same bits, and the tree is fixed: the result does not depend on
// timing.
template <int G, int N>
__device__ __forceinline__ void group_sum(double (&acc)[N]) {
#pragma unroll
    for (int c = 0; c < N; ++c) {
        if (G >= 2) acc[c] = __dadd_rn(acc[c], dpp_f64<0xB1>(acc[c]));    // quad_perm [1,0,3,2]
        if (G >= 4) acc[c] = __dadd_rn(acc[c], dpp_f64<0x4E>(acc[c]));    // quad_perm [2,3,0,1]
        if (G >= 8) acc[c] = __dadd_rn(acc[c], dpp_f64<0x141>(acc[c]));   // row_half_mirror
        if (G >= 16) acc[c] = __dadd_rn(acc[c], dpp_f64<0x140>(acc[c]));  // row_mirror
        if (G >= 32) acc[c] = __dadd_rn(acc[c], __shfl_xor(acc[c], 16, 64));
        if (G >= 64) acc[c] = __dadd_rn(acc[c], __shfl_xor(acc[c], 32, 64));
    }
}

// Accumulate one particle's restriction weights: PIT per leaf corner, PIDT
// per stencil slot of the owning vertex.
template <int D, int SCHEME, bool REG, int NS>
__device__ __forceinline__ void deposit_one(const DevInst &in, const double *xp, int e, double s, uint32_t su,
                                            double rinv, double qp, bool use_q, double (&acc)[NS]) {
    uint32_t bad = 0;
    Axis ax[D];
    uint32_t a[D];
    double f[D], g[D];
    if (REG && SCHEME == PIC_PIT) {
        // the stored positions lie in [0,1), so the cell is floor(y) and
        // f = y - floor(y) is y - I exactly, without the integer cell
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double y = __dmul_rn(xp[k], in.Sd);
            f[k] = __dsub_rn(y, floor(y));
            g[k] = __dsub_rn(1.0, f[k]);
        }
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            ax[k] = scale_axis(xp[k], in.Sd, in.S, bad);
            const uint32_t I = ax[k].T >> 1;
            a[k] = REG ? I : div_pow3(I, e);
            f[k] = REG ? __dsub_rn(ax[k].y, (double)I) : __dmul_rn(__dsub_rn(ax[k].y, (double)a[k] * s), rinv);
            g[k] = __dsub_rn(1.0, f[k]);
        }
    }
    if (SCHEME == PIC_PIT) {
#pragma unroll
        for (int c = 0; c < (1 << D); ++c) {
            double wc = (c & 1) ? f[0] : g[0];
#pragma unroll
            for (int k = 1; k < D; ++k) wc = __dmul_rn(wc, ((c >> k) & 1) ? f[k] : g[k]);
            acc[c] = __dadd_rn(acc[c], use_q ? __dmul_rn(qp, wc) : wc);
        }
    } else {
        // The owner is the corner nearest to the particle.  Per axis the
        // particle's two corner weights (g, f) land on stencil offsets {0,+1}
        // (owner below) or {-1,0} (owner above); the 3^d slot weights are the
        // tensor product of these per-axis triples, so every slot is updated
        // branch-free (absent ones with +0).
        double u[D][3];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const bool up = ax[k].T >= (2u * a[k] + 1u) * su;
            u[k][0] = up ? g[k] : 0.0;
            u[k][1] = up ? f[k] : g[k];
            u[k][2] = up ? 0.0 : f[k];
        }
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) {
            double wc = u[0][sl % 3];
            wc = __dmul_rn(wc, u[1][(sl / 3) % 3]);
            if (D == 3) wc = __dmul_rn(wc, u[D - 1][sl / 9]);
            acc[sl] = __dadd_rn(acc[sl], use_q ? __dmul_rn(qp, wc) : wc);
        }
    }
}

// G lanes per bin (64/G bins per wavefront).  A bin's particles are taken in
// batches of G*K; all loads of a batch are issued before the first is used,
// so a bin of up to G*K particles costs one memory latency after its offsets
// arrive.  With per-particle charges the terms are q_p w_c, otherwise w_c
// (the uniform charge is applied per vertex).
template <int D, int SCHEME, bool REG, int G, int K>
struct DepositBin {
    static constexpr int NS = SCHEME == PIC_PIT ? (1 << D) : (D == 2 ? 9 : 27);
    const DevInst *in;
    int e;
    double s, rinv;
    uint32_t su;
    int64_t p0, p1;

    __device__ __forceinline__ void setup(const DevTree &t, const DevInst &in0, const int64_t *bin_start, int64_t n,
                                          int64_t b, int lane) {
        int ii = 0;
        if (t.n_inst > 1) ii = SCHEME == PIC_PIT ? t.leaf_inst[b] : t.pidt_inst[b];
        in = t.n_inst > 1 ? &t.inst[ii] : &in0;
        const int lev = REG ? in->L : (SCHEME == PIC_PIT ? t.leaf_level[b] : t.pidt_level[b]);
        e = in->L - lev;
        s = (double)pow3_u32(e);
        su = pow3_u32(e);
        rinv = in->rinv[lev];
        p0 = ld_const(bin_start, (uint32_t)b);
        p1 = ld_const(bin_start, (uint32_t)b + 1u);
        if (p0 < 0 || p1 > n || p0 > p1) {             // malformed offsets: flag, touch nothing
            if (lane == 0) flag_status(t.status, PIC_DEV_RANGE);
            p0 = p1 = 0;
        }
    }
    // one batch of G*K particles from `base`: loads, then weights
    __device__ __forceinline__ void load(const F64Ptrs &P, const double *q, int64_t base, int lane, double (&xs)[K][D],
                                         double (&qs)[K]) const {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int64_t p = base + lane + G * k;
            const bool ok = p < p1;
#pragma unroll
            for (int d = 0; d < D; ++d) xs[k][d] = ok ? P.x[d][p] : 0.0;
            qs[k] = (ok && q) ? q[p] : 1.0;
        }
    }
    __device__ __forceinline__ void add(const double (&xs)[K][D], const double (&qs)[K], const double *q, int64_t base,
                                        int lane, double (&acc)[NS]) const {
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (base + lane + G * k < p1)
                deposit_one<D, SCHEME, REG, NS>(*in, xs[k], e, s, su, rinv, qs[k], q != nullptr, acc);
    }
};

// G lanes per bin (64/G bins per wavefront), BPW bins per group one after
// the other.  A bin's particles are taken in batches of G*K; when the group's
// bins each fit one batch, every load of all of them is issued before the
// first is used, so the group waits for memory once.  With per-particle
// charges the terms are q_p w_c, otherwise w_c (the uniform charge is applied
// per vertex).
template <int D, int SCHEME, bool REG, int G, int K, int BPW>
__global__ __launch_bounds__(256) void k_deposit_bins(DevTree t, DevInst in0, F64Ptrs P, int64_t n,
                                                      const int64_t *bin_start, int64_t n_bins, const double *q,
                                                      double *partial) {
    using DB = DepositBin<D, SCHEME, REG, G, K>;
    constexpr int NS = DB::NS;
    const int lane = threadIdx.x & (G - 1);
    const int64_t groups = (int64_t)gridDim.x * (blockDim.x / G);
    const int64_t g0 = (int64_t)blockIdx.x * (blockDim.x / G) + (threadIdx.x / G);
    for (int64_t b0 = g0 * BPW; b0 < n_bins; b0 += groups * BPW) {
        DB bin[BPW];
        bool one_batch = true;
#pragma unroll
        for (int i = 0; i < BPW; ++i) {
            const int64_t b = min(b0 + i, n_bins - 1);
            bin[i].setup(t, in0, bin_start, n, b, lane);
            if (b0 + i >= n_bins) bin[i].p1 = bin[i].p0;   // past the end: empty
            one_batch &= bin[i].p1 - bin[i].p0 <= (int64_t)G * K;
        }
        double acc[BPW][NS];
#pragma unroll
        for (int i = 0; i < BPW; ++i)
#pragma unroll
            for (int c = 0; c < NS; ++c) acc[i][c] = 0.0;
        if (one_batch) {
            double xs[BPW][K][D], qs[BPW][K];
#pragma unroll
            for (int i = 0; i < BPW; ++i) bin[i].load(P, q, bin[i].p0, lane, xs[i], qs[i]);
#pragma unroll
            for (int i = 0; i < BPW; ++i) bin[i].add(xs[i], qs[i], q, bin[i].p0, lane, acc[i]);
        } else {
#pragma unroll
            for (int i = 0; i < BPW; ++i)
                for (int64_t base = bin[i].p0; base < bin[i].p1; base += G * K) {
                    double xs[K][D], qs[K];
                    bin[i].load(P, q, base, lane, xs, qs);
                    bin[i].add(xs, qs, q, base, lane, acc[i]);
                }
        }
#pragma unroll
        for (int i = 0; i < BPW; ++i) {
            group_sum<G, NS>(acc[i]);
            if (lane == 0 && b0 + i < n_bins) {
#pragma unroll
                for (int c = 0; c < NS; ++c) partial[(b0 + i) * NS + c] = acc[i][c];
            }
        }
    }
}

// Per vertex: sum the partials of every (bin, slot) that lands on it, in a
// fixed order.  Regular instances enumerate them arithmetically, adaptive ones
// through the CSR incidence lists.
template <int D, int SCHEME, bool REG>
__global__ __launch_bounds__(256) void k_deposit_vertices(DevTree t, DevInst in0, const double *partial,
                                                          int64_t n_vtx, int use_q, double q_uniform, double *rho) {
    constexpr int NS = SCHEME == PIC_PIT ? (1 << D) : (D == 2 ? 9 : 27);
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n_vtx; v += (int64_t)gridDim.x * blockDim.x) {
        double sum = 0.0;
        const DevInst &in = t.n_inst > 1 ? t.inst[t.vtx_inst[v]] : in0;
        if (REG || in.regular) {
            const uint32_t S = (uint32_t)in.S;
            uint32_t J[D];
            uint32_t r = (uint32_t)(v - in.vtx_off);
#pragma unroll
            for (int k = 0; k < D; ++k) {
                J[k] = r % S;
                r /= S;
            }
            bool first = true;
            if (SCHEME == PIC_PIT) {
#pragma unroll
                for (int c = 0; c < (1 << D); ++c) {
                    uint32_t cell[D];
#pragma unroll
                    for (int k = 0; k < D; ++k) cell[k] = ((c >> k) & 1) ? (J[k] == 0 ? S - 1 : J[k] - 1) : J[k];
                    const int64_t leaf = in.leaf_off + regular_rank<D, REG>(t, in, cell);
                    const double x = partial[leaf * NS + c];
                    sum = first ? x : __dadd_rn(sum, x);
                    first = false;
                }
            } else {
                const uint32_t half = (S - 1u) >> 1;
#pragma unroll
                for (int sl = 0; sl < NS; ++sl) {
                    // owner B = J - o with o = digit - 1; its slot for vertex J is sl
                    uint32_t sh[D];
                    int z = sl;
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        const int o = z % 3 - 1;
                        z /= 3;
                        uint32_t B = J[k] + S - (uint32_t)(o + 1) + 1u;   // J - o + S
                        B = B >= S ? B - S : B;
                        B = B >= S ? B - S : B;
                        uint32_t Jp = B + half;
                        sh[k] = Jp >= S ? Jp - S : Jp;
                    }
                    const int64_t bin = in.pidt_off + regular_rank<D, REG>(t, in, sh);
                    const double x = partial[bin * NS + sl];
                    sum = first ? x : __dadd_rn(sum, x);
                    first = false;
                }
            }
        } else {
            const int32_t *ptr = SCHEME == PIC_PIT ? t.vinc_ptr : t.vpinc_ptr;
            const int32_t *lst = SCHEME == PIC_PIT ? t.vinc : t.vpinc;
            const int32_t j0 = ptr[v], j1 = ptr[v + 1];
            for (int32_t j = j0; j < j1; ++j) sum = j == j0 ? partial[lst[j]] : __dadd_rn(sum, partial[lst[j]]);
        }
        rho[v] = use_q ? sum : __dmul_rn(q_uniform, sum);
    }
}

__global__ void k_status_clear(uint32_t *status) { *status = 0; }

// Explicit Euler step with reflecting walls over SoA particle arrays.
template <int D>
__global__ __launch_bounds__(256) void k_stream_push(F64Ptrs P, int64_t n, double dt) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            double x = P.x[k][p], v = P.v[k][p];
            x = __dadd_rn(x, __dmul_rn(v, dt));
            if (x < 0.0) { x = -x; v = -v; }
            if (x > 1.0) { x = __dsub_rn(2.0, x); v = -v; }
            P.x[k][p] = x;
            P.v[k][p] = v;
        }
    }
}

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
    // lane's cell (two passes), per-lane loads for the rest
    float Ec[1 << D][D];
    uint64_t pend = __ballot(1);
    const uint32_t lane = __lane_id();
#pragma unroll
    for (int it = 0; it < 2; ++it) {
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
// bin is implicit in the segment it is stored in).  Clears the per-call
// counters.
template <int D, int SCHEME, bool MULTI>
__global__ __launch_bounds__(256) void k_step_key_f32(DevTree t, DevInst in0, F32Ptrs P, int64_t n, double qmdt0,
                                                      double dt0, const double *qa, const double *da,
                                                      const int64_t *inst_start, const int64_t *bin_start,
                                                      uint32_t n_bins, const uint32_t *tile_bin, int tile,
                                                      uint32_t *key_out, const uint32_t *wave_bin) {
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
        const uint32_t ob = old_bin_wave(bin_start, n_bins, tile_bin, tile, p, wave_bin);
        uint32_t c[D];
        cell_of<D, SCHEME>(t, in, local_rank<SCHEME>(in, ob, bad), o, c);
        uint32_t nb = push_f32<D, SCHEME>(t, in, P, c, o, u, kick, bad);
        if (nb >= n_bins) bad |= PIC_DEV_RANGE;
        nb = min(nb, n_bins - 1u);
        key_out[p] = 2u * nb + (nb == ob ? 0u : 1u);
        if (bad) flag_status(t.status, bad);
    }
}

// FP32 form, emit pass of pic_step: the state pushed again is staged through
// LDS in tile-sorted order, one column at a time, and written run by run (as
// k_step_emit).
template <int D, int SCHEME, bool MULTI, int TILE, int NT>
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
        if (p >= n) continue;
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

// ----------------------------------------------------------------- launchers

static int grid_for(int64_t items, int per_block, int cap) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

static F64Ptrs make_ptrs(const pic_tree *t, const pic_particles *p, const double *const *E, double *Ep) {
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

#define PIC_DISPATCH_GP(D, SCH, REG, MULTI)                                                              \
    PIC_LAUNCH("gather_push", (k_gather_push<D, SCH, REG, MULTI>), dim3(grid), dim3(256), 0, s, t->dt, t->inst0, P, \
                       p->n, qmdt, dt, qa, da, p->inst_start_dev, bin)

hipError_t launch_gather_push(const pic_tree *t, int scheme, pic_particles *p, const double *const *E,
                              double qmdt, double dt, const pic_push_params *pp, uint32_t *bin,
                              double *Ep, hipStream_t s) {
    if (p->n == 0) return hipSuccess;
    F64Ptrs P = make_ptrs(t, p, E, Ep);
    const double *qa = pp ? pp->qmdt_dev : nullptr;
    const double *da = pp ? pp->dt_dev : nullptr;
    const int grid = grid_for(p->n, 256, 1 << 20);
    const bool multi = t->n_inst > 1;
    const bool reg = t->reg_kernels != 0;
    if (t->dim == 2) {
        if (scheme == PIC_PIT) {
            if (multi) { if (reg) PIC_DISPATCH_GP(2, 0, true, true); else PIC_DISPATCH_GP(2, 0, false, true); }
            else { if (reg) PIC_DISPATCH_GP(2, 0, true, false); else PIC_DISPATCH_GP(2, 0, false, false); }
        } else {
            if (multi) { if (reg) PIC_DISPATCH_GP(2, 1, true, true); else PIC_DISPATCH_GP(2, 1, false, true); }
            else { if (reg) PIC_DISPATCH_GP(2, 1, true, false); else PIC_DISPATCH_GP(2, 1, false, false); }
        }
    } else {
        if (scheme == PIC_PIT) {
            if (multi) { if (reg) PIC_DISPATCH_GP(3, 0, true, true); else PIC_DISPATCH_GP(3, 0, false, true); }
            else { if (reg) PIC_DISPATCH_GP(3, 0, true, false); else PIC_DISPATCH_GP(3, 0, false, false); }
        } else {
            if (multi) { if (reg) PIC_DISPATCH_GP(3, 1, true, true); else PIC_DISPATCH_GP(3, 1, false, true); }
            else { if (reg) PIC_DISPATCH_GP(3, 1, true, false); else PIC_DISPATCH_GP(3, 1, false, false); }
        }
    }
    return hipGetLastError();
}

#define PIC_DISPATCH_LOC(D, SCH, REG, MULTI)                                                           \
    PIC_LAUNCH("locate", (k_locate<D, SCH, REG, MULTI>), dim3(grid), dim3(256), 0, s, t->dt, t->inst0, P, p->n, \
                       p->inst_start_dev, bin)

hipError_t launch_locate(const pic_tree *t, int scheme, const pic_particles *p, uint32_t *bin, hipStream_t s) {
    if (p->n == 0) return hipSuccess;
    F64Ptrs P = make_ptrs(t, p, nullptr, nullptr);
    const int grid = grid_for(p->n, 256, 1 << 20);
    const bool multi = t->n_inst > 1;
    const bool reg = t->reg_kernels != 0;
    if (t->dim == 2) {
        if (scheme == PIC_PIT) {
            if (multi) { if (reg) PIC_DISPATCH_LOC(2, 0, true, true); else PIC_DISPATCH_LOC(2, 0, false, true); }
            else { if (reg) PIC_DISPATCH_LOC(2, 0, true, false); else PIC_DISPATCH_LOC(2, 0, false, false); }
        } else {
            if (multi) { if (reg) PIC_DISPATCH_LOC(2, 1, true, true); else PIC_DISPATCH_LOC(2, 1, false, true); }
            else { if (reg) PIC_DISPATCH_LOC(2, 1, true, false); else PIC_DISPATCH_LOC(2, 1, false, false); }
        }
    } else {
        if (scheme == PIC_PIT) {
            if (multi) { if (reg) PIC_DISPATCH_LOC(3, 0, true, true); else PIC_DISPATCH_LOC(3, 0, false, true); }
            else { if (reg) PIC_DISPATCH_LOC(3, 0, true, false); else PIC_DISPATCH_LOC(3, 0, false, false); }
        } else {
            if (multi) { if (reg) PIC_DISPATCH_LOC(3, 1, true, true); else PIC_DISPATCH_LOC(3, 1, false, true); }
            else { if (reg) PIC_DISPATCH_LOC(3, 1, true, false); else PIC_DISPATCH_LOC(3, 1, false, false); }
        }
    }
    return hipGetLastError();
}

static int64_t n_bins_of(const pic_tree *t, int scheme) {
    return scheme == PIC_PIT ? t->leaf_off.back() : t->pidt_off.back();
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct RebinLayout {
    size_t tile_bin, perm, run_key, run_info, run_dest, tile_nruns, key_cnt, key_nruns, key_fill, key_cn, key_base,
        list_off,
        list, scan_state, scan_ctr, khead, run_wcnt, meta, keys, klist, knext, wave_bin, total;
};

static RebinLayout rebin_layout(int64_t n, int64_t n_bins, int tile) {
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
    L.klist = o; o = align256(o + keys * KLIST_CAP * 4);
    L.knext = o; o = align256(o + slots * 4);
    L.wave_bin = o; o = align256(o + (slots / 64 + 1) * 4);
    L.total = o;
    return L;
}

Tuning g_tune;

size_t rebin_scratch_bytes(const pic_tree *t, int64_t n, int scheme) {
    // large enough for every supported tile size
    const int64_t nb = n_bins_of(t, scheme);
    return std::max({rebin_layout(n, nb, 1024).total, rebin_layout(n, nb, 2048).total, rebin_layout(n, nb, 4096).total});
}

template <int IPT>
static void launch_tiles(int radix, dim3 g, hipStream_t s, const uint32_t *nb, const int64_t *os, int64_t n,
                         uint32_t n_bins, const RebinScratch &sc, uint32_t *status) {
    if (radix == 5) PIC_LAUNCH("rebin_tiles", (k_rebin_tiles<IPT, 5>), g, dim3(RB_THREADS), 0, s, nb, os, n, n_bins, sc, status);
    else PIC_LAUNCH("rebin_tiles", (k_rebin_tiles<IPT, 4>), g, dim3(RB_THREADS), 0, s, nb, os, n, n_bins, sc, status);
}

template <int IPT, int MODE, bool NT>
static void launch_scatter_g(dim3 g, hipStream_t s, int64_t n, const RebinScratch &sc, const Cols &cols,
                             uint32_t *status) {
    switch (g_tune.scatter_group) {
        case 1: PIC_LAUNCH("rebin_scatter", (k_rebin_scatter<IPT, MODE, NT, 1>), g, dim3(RB_THREADS), 0, s, n, sc, cols, status); break;
        case 2: PIC_LAUNCH("rebin_scatter", (k_rebin_scatter<IPT, MODE, NT, 2>), g, dim3(RB_THREADS), 0, s, n, sc, cols, status); break;
        default: PIC_LAUNCH("rebin_scatter", (k_rebin_scatter<IPT, MODE, NT, 4>), g, dim3(RB_THREADS), 0, s, n, sc, cols, status); break;
    }
}

template <int IPT>
static void launch_scatter(int mode, dim3 g, hipStream_t s, int64_t n, const RebinScratch &sc, const Cols &cols,
                           uint32_t *status) {
    const bool nt = g_tune.scatter_nt != 0;
    if (mode == 1) {
        if (nt) launch_scatter_g<IPT, 1, true>(g, s, n, sc, cols, status);
        else launch_scatter_g<IPT, 1, false>(g, s, n, sc, cols, status);
    } else {
        if (nt) launch_scatter_g<IPT, 0, true>(g, s, n, sc, cols, status);
        else launch_scatter_g<IPT, 0, false>(g, s, n, sc, cols, status);
    }
}

static RebinScratch bind_scratch(const RebinLayout &L, char *base) {
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
    return sc;
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

// The middle of the fused step: scan, then placement from the per-key lists.
static void launch_step_middle(const pic_tree *t, int64_t n, int64_t n_bins, const RebinScratch &sc,
                               int64_t *new_start, hipStream_t s) {
    const int64_t keys = 2 * n_bins;
    PIC_LAUNCH("step_scan", k_step_scan, dim3((keys + SP_KEYS - 1) / SP_KEYS), dim3(SP_THREADS), 0, s, (uint32_t)keys,
               (uint32_t)n_bins, n, sc, new_start, t->dt.status);
    if (n > 0)
        PIC_LAUNCH("step_place", k_step_place, dim3(grid_for(keys, 16, 1 << 16)), dim3(256), 0, s, sc, (uint32_t)keys);
}

hipError_t launch_rebin(const pic_tree *t, int scheme, int64_t n, const uint32_t *new_bin, const int64_t *old_start,
                        const Cols &cols, int64_t *new_start, void *scratch, size_t scratch_bytes, hipStream_t s) {
    const int64_t n_bins = n_bins_of(t, scheme);
    const int ipt = g_tune.rebin_ipt;
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
        if (ipt == 8) launch_tiles<8>(g_tune.rebin_radix, dim3(tiles), s, new_bin, old_start, n, (uint32_t)n_bins, sc, t->dt.status);
        else launch_tiles<16>(g_tune.rebin_radix, dim3(tiles), s, new_bin, old_start, n, (uint32_t)n_bins, sc, t->dt.status);
    }
    launch_rebin_middle(t, n, n_bins, tile, sc, new_start, s);
    if (n > 0) {
        if (ipt == 8) launch_scatter<8>(g_tune.scatter_mode, dim3(tiles), s, n, sc, cols, t->dt.status);
        else launch_scatter<16>(g_tune.scatter_mode, dim3(tiles), s, n, sc, cols, t->dt.status);
    }
    return hipGetLastError();
}

size_t deposit_scratch_bytes(const pic_tree *t, int scheme);
hipError_t launch_deposit(const pic_tree *t, int scheme, const pic_particles *p, const int64_t *bin_start,
                          const double *q, double q_uniform, double *rho, void *scratch, size_t scratch_bytes,
                          hipStream_t s);

struct StepArgs {
    uint32_t *zero;   // per-call counters, cleared by the first pass when it can
    int64_t n_zero;
    F64Ptrs P, out;
    int64_t n;
    double qmdt, dt;
    const double *qa, *da;
    const int64_t *inst_start, *old_start;
    uint32_t n_bins;
};

#define PIC_EMIT(NT, ST)                                                                                      \
    PIC_LAUNCH("step_emit", (k_step_emit<D, SCH, REG, MULTI, TILE, NT, ST>), dim3(tiles), dim3(NT), 0, s, t->dt,  \
               t->inst0, a.P, a.n, a.qmdt, a.dt, a.qa, a.da, a.inst_start, (const uint32_t *)sc.meta,          \
               (const uint32_t *)sc.run_dest, (const uint32_t *)sc.run_info, a.out, extra, g_tune.xcd_tiles)

template <int D, int SCH, bool REG, bool MULTI, int TILE>
static void launch_emit(const pic_tree *t, const StepArgs &a, const RebinScratch &sc, const Cols &extra,
                        int64_t tiles, hipStream_t s) {
    const int st = g_tune.emit_stage;
    if (g_tune.emit_threads == 1024) {
        if (st == 2) PIC_EMIT(1024, 2); else if (st == 1) PIC_EMIT(1024, 1); else PIC_EMIT(1024, 0);
    } else if (g_tune.emit_threads == 512) {
        if (st == 2) PIC_EMIT(512, 2); else if (st == 1) PIC_EMIT(512, 1); else PIC_EMIT(512, 0);
    } else {
        if (st == 2) PIC_EMIT(256, 2); else if (st == 1) PIC_EMIT(256, 1); else PIC_EMIT(256, 0);
    }
}

template <int D, int SCH, bool REG, bool MULTI, int IPT>
static void launch_step_passes(const pic_tree *t, const StepArgs &a, const RebinScratch &sc, const Cols &extra,
                               int64_t *new_start, hipStream_t s) {
    const int64_t tiles = (a.n + StepShape<IPT>::TILE - 1) / StepShape<IPT>::TILE;
    if (g_tune.step_rank) {
        if (a.n > 0 && g_tune.step_rank == 2) {
            PIC_LAUNCH("step_key", (k_step_key<D, SCH, REG, MULTI>), dim3(grid_for(a.n, 256, 1 << 20)), dim3(256), 0,
                       s, t->dt, t->inst0, a.P, a.n, a.qmdt, a.dt, a.qa, a.da, a.inst_start, a.old_start, a.n_bins,
                       sc.keys, a.zero, a.n_zero);
            PIC_LAUNCH("step_group", (k_step_group<IPT>), dim3(tiles), dim3(RB_THREADS), 0, s,
                       (const uint32_t *)sc.keys, a.n, sc, sc.meta, 0);
        } else if (a.n > 0) {
            PIC_LAUNCH("step_rank", (k_step_rank<D, SCH, REG, MULTI, IPT>), dim3(tiles), dim3(RB_THREADS), 0, s,
                       t->dt, t->inst0, a.P, a.n, a.qmdt, a.dt, a.qa, a.da, a.inst_start, a.old_start, a.n_bins, sc,
                       sc.meta, 0);
        }
        launch_step_middle(t, a.n, a.n_bins, sc, new_start, s);
        if (a.n > 0) launch_emit<D, SCH, REG, MULTI, StepShape<IPT>::TILE>(t, a, sc, extra, tiles, s);
        return;
    }
    if (a.n > 0)
        PIC_LAUNCH("step_count", (k_step_count<D, SCH, REG, MULTI, IPT>), dim3(tiles), dim3(RB_THREADS), 0, s,
                   t->dt, t->inst0, a.P, a.n, a.qmdt, a.dt, a.qa, a.da, a.inst_start, a.old_start, a.n_bins, sc);
    launch_rebin_middle(t, a.n, a.n_bins, StepShape<IPT>::TILE, sc, new_start, s);
    if (a.n > 0)
        PIC_LAUNCH("step_move", (k_step_move<D, SCH, REG, MULTI, IPT>), dim3(tiles), dim3(RB_THREADS), 0, s, t->dt,
                   t->inst0, a.P, a.n, a.qmdt, a.dt, a.qa, a.da, a.inst_start, a.old_start, a.n_bins, sc, a.out,
                   extra);
}

template <int D, int SCH, bool REG, bool MULTI>
static void launch_step_ipt(const pic_tree *t, const StepArgs &a, const RebinScratch &sc, const Cols &extra,
                            int64_t *new_start, hipStream_t s) {
    if (g_tune.step_ipt == 4) launch_step_passes<D, SCH, REG, MULTI, 4>(t, a, sc, extra, new_start, s);
    else launch_step_passes<D, SCH, REG, MULTI, 8>(t, a, sc, extra, new_start, s);
}

template <int D, int SCH>
static void launch_step_shape(const pic_tree *t, const StepArgs &a, const RebinScratch &sc, const Cols &extra,
                              int64_t *new_start, hipStream_t s) {
    const bool multi = t->n_inst > 1, reg = t->reg_kernels != 0;
    if (multi) {
        if (reg) launch_step_ipt<D, SCH, true, true>(t, a, sc, extra, new_start, s);
        else launch_step_ipt<D, SCH, false, true>(t, a, sc, extra, new_start, s);
    } else {
        if (reg) launch_step_ipt<D, SCH, true, false>(t, a, sc, extra, new_start, s);
        else launch_step_ipt<D, SCH, false, false>(t, a, sc, extra, new_start, s);
    }
}

hipError_t launch_step(const pic_tree *t, int scheme, pic_particles *in, const int64_t *old_start,
                       const double *const *E, double qmdt, double dt, const pic_push_params *pp, const Cols &extra,
                       pic_particles *out, int64_t *new_start, int q_col, double q_uniform, double *rho,
                       void *scratch, size_t scratch_bytes, hipStream_t s) {
    const int64_t n = in->n;
    const int64_t n_bins = n_bins_of(t, scheme);
    const int tile = RB_THREADS * g_tune.step_ipt;
    const RebinLayout L = rebin_layout(n, n_bins, tile);
    if (scratch_bytes < L.total || scratch_bytes < deposit_scratch_bytes(t, scheme)) return hipErrorInvalidValue;
    char *base = (char *)scratch;
    const RebinScratch sc = bind_scratch(L, base);
    const int64_t zero_words = (int64_t)((L.key_base - L.key_cnt) / 4);
    StepArgs a;
    a.zero = (uint32_t *)(base + L.key_cnt);
    a.n_zero = zero_words;
    // the key pass of the three-pass form clears the counters itself
    if (!(g_tune.step_rank == 2 && n > 0))
        PIC_LAUNCH("rebin_prep", k_rebin_prep, dim3(grid_for(zero_words, 256, 4096)), dim3(256), 0, s,
                   (uint32_t *)(base + L.key_cnt), zero_words, nullptr, n_bins, n, tile, sc);
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

size_t deposit_scratch_bytes(const pic_tree *t, int scheme) {
    const int ns = scheme == PIC_PIT ? (1 << t->dim) : (t->dim == 2 ? 9 : 27);
    return align256((size_t)n_bins_of(t, scheme) * ns * sizeof(double));
}

#define PIC_DEP_BINS(D, SCH, REG, G)                                                                          \
    do {                                                                                                      \
        if (g_tune.deposit_bpw == 2)                                                                          \
            PIC_LAUNCH("deposit_bins", (k_deposit_bins<D, SCH, REG, G, 256 / G, 2>),                          \
                       dim3(grid_for((n_bins + 1) / 2, 256 / G, 1 << 18)), dim3(256), 0, s, t->dt, t->inst0, P, p->n, \
                       bin_start, n_bins, q, partial);                                                        \
        else                                                                                                  \
            PIC_LAUNCH("deposit_bins", (k_deposit_bins<D, SCH, REG, G, 256 / G, 1>),                          \
                       dim3(grid_for(n_bins, 256 / G, 1 << 18)), dim3(256), 0, s, t->dt, t->inst0, P, p->n,   \
                       bin_start, n_bins, q, partial);                                                        \
    } while (0)

#define PIC_DISPATCH_DEP(D, SCH, REG)                                                                         \
    do {                                                                                                     \
        if (g_tune.deposit_lanes == 16) PIC_DEP_BINS(D, SCH, REG, 16);                                       \
        else if (g_tune.deposit_lanes == 32) PIC_DEP_BINS(D, SCH, REG, 32);                                  \
        else PIC_DEP_BINS(D, SCH, REG, 64);                                                                  \
        PIC_LAUNCH("deposit_vertices", (k_deposit_vertices<D, SCH, REG>), dim3(grid_for(n_vtx, 256, 1 << 16)), dim3(256), \
                           0, s, t->dt, t->inst0, partial, n_vtx, q ? 1 : 0, q_uniform, rho);                 \
    } while (0)

hipError_t launch_deposit(const pic_tree *t, int scheme, const pic_particles *p, const int64_t *bin_start,
                          const double *q, double q_uniform, double *rho, void *scratch, size_t scratch_bytes,
                          hipStream_t s) {
    const int64_t n_bins = n_bins_of(t, scheme);
    const int64_t n_vtx = t->vtx_off.back();
    if (scratch_bytes < deposit_scratch_bytes(t, scheme)) return hipErrorInvalidValue;
    double *partial = (double *)scratch;
    F64Ptrs P = make_ptrs(t, p, nullptr, nullptr);
    const bool reg = t->reg_kernels != 0;
    if (t->dim == 2) {
        if (scheme == PIC_PIT) { if (reg) PIC_DISPATCH_DEP(2, 0, true); else PIC_DISPATCH_DEP(2, 0, false); }
        else { if (reg) PIC_DISPATCH_DEP(2, 1, true); else PIC_DISPATCH_DEP(2, 1, false); }
    } else {
        if (scheme == PIC_PIT) { if (reg) PIC_DISPATCH_DEP(3, 0, true); else PIC_DISPATCH_DEP(3, 0, false); }
        else { if (reg) PIC_DISPATCH_DEP(3, 1, true); else PIC_DISPATCH_DEP(3, 1, false); }
    }
    return hipGetLastError();
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
    PIC_LAUNCH("deposit_vertices", (k_deposit_vertices<D, SCH, true>), dim3(grid_for(n_vtx, 256, 1 << 16)), dim3(256),
               0, s, t->dt, t->inst0, partial, n_vtx, q ? 1 : 0, q_uniform, rho);
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
                            hipStream_t s) {
    constexpr int TILE = 2048;
    const int64_t tiles = (n + TILE - 1) / TILE;
    PIC_LAUNCH("step_key_f32", (k_step_key_f32<D, SCH, MULTI>), dim3(grid_for(n, 256, 1 << 20)), dim3(256), 0, s,
               t->dt, t->inst0, P, n, qmdt, dt, qa, da, inst_start, old_start, n_bins, (const uint32_t *)sc.tile_bin,
               TILE, sc.keys, (const uint32_t *)sc.wave_bin);
    PIC_LAUNCH("step_group", (k_step_group<8>), dim3(tiles), dim3(RB_THREADS), 0, s, (const uint32_t *)sc.keys, n, sc,
               sc.meta, 0);
    launch_step_middle(t, n, n_bins, sc, new_start, s);
    PIC_LAUNCH("step_emit_f32", (k_step_emit_f32<D, SCH, MULTI, TILE, 1024>), dim3(tiles), dim3(1024), 0, s, t->dt,
               t->inst0, P, n, qmdt, dt, qa, da, inst_start, old_start, n_bins, (const uint32_t *)sc.tile_bin,
               (const uint32_t *)sc.meta, (const uint32_t *)sc.run_dest, (const uint32_t *)sc.run_info, Q, extra,
               g_tune.xcd_tiles, (const uint32_t *)sc.wave_bin);
}

hipError_t launch_step_f32(const pic_tree *t, int scheme, pic_particles *in, const int64_t *old_start,
                           const double *const *E, double qmdt, double dt, const pic_push_params *pp,
                           const Cols &extra, pic_particles *out, int64_t *new_start, int q_col, double q_uniform,
                           double *rho, void *scratch, size_t scratch_bytes, hipStream_t s) {
    const int64_t n = in->n;
    const int64_t n_bins = n_bins_of(t, scheme);
    if (scratch_bytes < step_f32_scratch_bytes(t, n, scheme)) return hipErrorInvalidValue;
    if (g_tune.step_rank != 0 && n > 0) {
        // key, group, scan, place and emit passes, as the FP64 step
        constexpr int TILE = 2048;
        const RebinLayout L = rebin_layout(n, n_bins, TILE);
        char *base = (char *)scratch;
        const RebinScratch sc = bind_scratch(L, base);
        const int64_t zero_words = (int64_t)((L.key_base - L.key_cnt) / 4);
        PIC_LAUNCH("rebin_prep", k_rebin_prep, dim3(grid_for(std::max(zero_words, n_bins), 256, 4096)), dim3(256), 0,
                   s, (uint32_t *)(base + L.key_cnt), zero_words, old_start, n_bins, n, TILE, sc);
        const F32Ptrs P = make_f32(t, in, E), Q = make_f32(t, out, E);
        const double *qa = pp ? pp->qmdt_dev : nullptr;
        const double *da = pp ? pp->dt_dev : nullptr;
        PIC_SWITCH_DSM(step_passes_f32, t, P, Q, n, qmdt, dt, qa, da, in->inst_start_dev, old_start,
                       (uint32_t)n_bins, sc, extra, new_start, s);
        const double *q = q_col >= 0 ? (const double *)extra.out[q_col] : nullptr;
        return launch_deposit_f32(t, scheme, out, new_start, q, q_uniform, rho, scratch, scratch_bytes, s);
    }
    const size_t rb = rebin_scratch_bytes(t, n, scheme);
    char *base = (char *)scratch;
    uint32_t *bins = (uint32_t *)(base + rb);
    const int tile = RB_THREADS * g_tune.rebin_ipt;
    const RebinLayout L = rebin_layout(n, n_bins, tile);
    const RebinScratch sc = bind_scratch(L, base);
    if (n > 0) {
        PIC_LAUNCH("rebin_prep", k_rebin_prep, dim3(grid_for(n_bins, 256, 4096)), dim3(256), 0, s, (uint32_t *)nullptr,
                   (int64_t)0, old_start, n_bins, n, tile, sc);
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

hipError_t launch_stream_push(int dim, int64_t n, double *const *x, double *const *v, double dt, hipStream_t s) {
    if (n == 0) return hipSuccess;
    F64Ptrs P{};
    for (int k = 0; k < dim; ++k) {
        P.x[k] = x[k];
        P.v[k] = v[k];
    }
    const int grid = grid_for(n, 256, 1 << 20);
    if (dim == 2) PIC_LAUNCH("stream_push", k_stream_push<2>, dim3(grid), dim3(256), 0, s, P, n, dt);
    else PIC_LAUNCH("stream_push", k_stream_push<3>, dim3(grid), dim3(256), 0, s, P, n, dt);
    return hipGetLastError();
}

hipError_t launch_status_clear(const pic_tree *t, hipStream_t s) {
    hipLaunchKernelGGL(k_status_clear, dim3(1), dim3(1), 0, s, t->dt.status);
    return hipGetLastError();
}

}  // namespace pic
