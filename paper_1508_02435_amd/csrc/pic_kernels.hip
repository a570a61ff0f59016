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
__device__ __forceinline__ int inst_of(const int64_t *start, int n_inst, int64_t p) {
    int lo = 0, hi = n_inst - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
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
            return (uint32_t)in.leaf_off + peano_low<D>(c, in.L);
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
            return (uint32_t)in.pidt_off + peano_low<D>(c, in.L);
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
        Axis ax[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            ax[k] = scale_axis(xv[k], in.Sd, in.S, bad);
            if (!(vv[k] - vv[k] == 0.0)) bad |= PIC_DEV_NONFINITE;
        }
        // leaf holding x: coordinates a, width s, corner vertex ids
        uint32_t I[D], a[D];
#pragma unroll
        for (int k = 0; k < D; ++k) I[k] = ax[k].T >> 1;
        int lev = in.L;
        int32_t vid[1 << D];
        if (REG) {
#pragma unroll
            for (int k = 0; k < D; ++k) a[k] = I[k];
            const uint32_t S = (uint32_t)in.S;
#pragma unroll
            for (int c = 0; c < (1 << D); ++c) {
                uint32_t idx = 0, m = 1;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    uint32_t j = I[k] + ((c >> k) & 1);
                    if (j >= S) j -= S;
                    idx += j * m;
                    m *= S;
                }
                vid[c] = in.vtx_off + (int32_t)idx;
            }
        } else {
            const uint32_t rank = descend<D>(t, in, I, lds, lds_n, lev);
#pragma unroll
            for (int k = 0; k < D; ++k) a[k] = div_pow3(I[k], in.L - lev);
#pragma unroll
            for (int c = 0; c < (1 << D); ++c) vid[c] = t.leaf_vtx[(int64_t)rank * (1 << D) + c];
        }
        const double s = (double)pow3_u32(in.L - lev);
        const double rinv = in.rinv[lev];
        double f[D], g[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            f[k] = __dmul_rn(__dsub_rn(ax[k].y, (double)a[k] * s), rinv);
            g[k] = __dsub_rn(1.0, f[k]);
        }
        double w[1 << D];
#pragma unroll
        for (int c = 0; c < (1 << D); ++c) {
            double wc = (c & 1) ? f[0] : g[0];
#pragma unroll
            for (int k = 1; k < D; ++k) wc = __dmul_rn(wc, ((c >> k) & 1) ? f[k] : g[k]);
            w[c] = wc;
        }
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const double *Ej = P.E[j];
            double e = __dmul_rn(w[0], Ej[vid[0]]);
#pragma unroll
            for (int c = 1; c < (1 << D); ++c) e = __dadd_rn(e, __dmul_rn(w[c], Ej[vid[c]]));
            if (P.Ep[0]) P.Ep[j][p] = e;
            double vj = __dadd_rn(vv[j], __dmul_rn(qmdt, e));
            double xj = __dadd_rn(xv[j], __dmul_rn(vj, dt));
            xj = __dsub_rn(xj, floor(xj));
            if (xj == 1.0) xj = 0.0;
            vv[j] = vj;
            xv[j] = xj;
        }
#pragma unroll
        for (int k = 0; k < D; ++k) {
            P.x[k][p] = xv[k];
            P.v[k][p] = vv[k];
        }
        uint32_t dummy = 0;
#pragma unroll
        for (int k = 0; k < D; ++k) ax[k] = scale_axis(xv[k], in.Sd, in.S, dummy);
        bad |= dummy;
        bin_out[p] = bin_of<D, SCHEME, REG>(t, in, ax, lds, lds_n);
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
constexpr int RB_IPT = 16;
constexpr int RB_TILE = RB_THREADS * RB_IPT;   // 4096 particles per tile
constexpr int RB_RADIX = 4;                    // bits per LDS radix pass
constexpr int RB_DIGITS = 1 << RB_RADIX;

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

struct RebinScratch {
    uint16_t *perm;       // n_tiles * TILE: tile-local source index per sorted slot
    uint32_t *run_key;    // n_tiles * TILE
    uint32_t *run_info;   // start | count << 16
    uint32_t *run_dest;   // n_tiles * TILE
    uint32_t *tile_nruns; // n_tiles
    uint32_t *key_cnt;    // 2*n_bins (zeroed per call)
    uint32_t *key_nruns;  // 2*n_bins (zeroed per call)
    uint32_t *key_fill;   // 2*n_bins (zeroed per call)
    uint32_t *key_base;   // 2*n_bins
    uint32_t *list_off;   // 2*n_bins + 1
    uint32_t *list;       // total runs <= n_tiles * TILE
    uint64_t *scan_state; // per scan block (zeroed per call)
    uint32_t *scan_ctr;   // dynamic block counter (zeroed per call)
};

// Pass 1: per tile, stable LDS radix sort of particle slots by key
// 2*bin + arrived, emitting runs of equal key.
__global__ __launch_bounds__(RB_THREADS) void k_rebin_tiles(const uint32_t *new_bin, const int64_t *old_start,
                                                           int64_t n, uint32_t n_bins, RebinScratch sc,
                                                           uint32_t *status) {
    __shared__ uint32_t s_key[RB_TILE];
    __shared__ uint16_t s_item[2][RB_TILE];
    __shared__ uint32_t s_cnt[RB_DIGITS * RB_THREADS + 1];   // +1: run-start sentinel
    __shared__ uint32_t s_wsum[4];
    __shared__ uint32_t s_misc[4];
    const int tid = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const int64_t lo = tile * RB_TILE;
    const int cnt = (int)min((int64_t)RB_TILE, n - lo);

    // old bin of each slot: the segment of old_start that holds it
    if (old_start) {
        for (int i = tid; i < RB_TILE; i += RB_THREADS) s_cnt[i] = 0;  // head counts (reuse)
        if (tid == 0) {
            // first bin b with old_start[b] <= lo < old_start[b+1]; last bin starting before lo+cnt
            int64_t a = 0, b = n_bins;  // upper_bound of lo in old_start[0..n_bins]
            while (a < b) {
                int64_t m = (a + b) >> 1;
                if (old_start[m] <= lo) a = m + 1; else b = m;
            }
            s_misc[0] = (uint32_t)(a - 1);
            int64_t hi = lo + cnt - 1;
            int64_t c = a > 0 ? a - 1 : 0, d = n_bins;   // a >= 1 unless the offsets are malformed
            while (c < d) {
                int64_t m = (c + d) >> 1;
                if (old_start[m] <= hi) c = m + 1; else d = m;
            }
            s_misc[1] = (uint32_t)c;  // bins in (first, c) start inside the tile
        }
        __syncthreads();
        const uint32_t b0 = s_misc[0], b1 = s_misc[1];
        for (uint32_t b = b0 + 1 + tid; b < b1; b += RB_THREADS) {
            const int64_t at = old_start[b] - lo;
            if (at >= 0 && at < cnt) atomicAdd(&s_cnt[(int)at], 1u);
        }
        __syncthreads();
        // inclusive scan of head counts: slot i lies in bin b0 + heads(<= i)
        uint32_t loc[RB_IPT];
        uint32_t sum = 0;
#pragma unroll
        for (int j = 0; j < RB_IPT; ++j) {
            sum += s_cnt[tid * RB_IPT + j];
            loc[j] = sum;
        }
        uint32_t tot;
        uint32_t base = block_excl_scan(sum, s_wsum, &tot);
#pragma unroll
        for (int j = 0; j < RB_IPT; ++j) {
            const int i = tid * RB_IPT + j;
            if (i < cnt) {
                uint32_t nb = new_bin[lo + i];
                if (nb >= n_bins) {
                    flag_status(status, PIC_DEV_RANGE);
                    nb = n_bins - 1;
                }
                const uint32_t ob = b0 + base + loc[j];
                s_key[i] = 2u * nb + (nb != ob ? 1u : 0u);
            }
        }
    } else {
        for (int i = tid; i < cnt; i += RB_THREADS) {
            uint32_t nb = new_bin[lo + i];
            if (nb >= n_bins) {
                flag_status(status, PIC_DEV_RANGE);
                nb = n_bins - 1;
            }
            s_key[i] = 2u * nb + 1u;
        }
    }
    __syncthreads();

    // key range of the tile -> number of radix passes
    uint32_t kmin = 0xffffffffu, kmax = 0;
    for (int i = tid; i < cnt; i += RB_THREADS) {
        kmin = min(kmin, s_key[i]);
        kmax = max(kmax, s_key[i]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        kmin = min(kmin, (uint32_t)__shfl_xor((int)kmin, o, 64));
        kmax = max(kmax, (uint32_t)__shfl_xor((int)kmax, o, 64));
    }
    if (tid == 0) { s_misc[2] = 0xffffffffu; s_misc[3] = 0; }
    __syncthreads();
    if ((tid & 63) == 0) {
        atomicMin(&s_misc[2], kmin);
        atomicMax(&s_misc[3], kmax);
    }
    __syncthreads();
    kmin = s_misc[2];
    kmax = s_misc[3];
    const uint32_t span = kmax - kmin;
    const int bits = span ? 32 - __clz(span) : 0;
    const int passes = (bits + RB_RADIX - 1) / RB_RADIX;

    for (int i = tid; i < RB_TILE; i += RB_THREADS) {
        if (i < cnt) s_key[i] -= kmin;
        s_item[0][i] = (uint16_t)i;
    }
    __syncthreads();

    // LSD radix passes: thread t owns the contiguous slots [t*IPT, (t+1)*IPT)
    // of the current order, so ranks within a digit follow slot order.
    int cur = 0;
    for (int ps = 0; ps < passes; ++ps) {
        const int shift = ps * RB_RADIX;
#pragma unroll
        for (int dg = 0; dg < RB_DIGITS; ++dg) s_cnt[dg * RB_THREADS + tid] = 0;
        uint8_t dig[RB_IPT], rk[RB_IPT];
        uint16_t it[RB_IPT];
#pragma unroll
        for (int j = 0; j < RB_IPT; ++j) {
            const int slot = tid * RB_IPT + j;
            it[j] = s_item[cur][slot];
            uint32_t dgt = RB_DIGITS - 1;                  // padding slots sort last
            if (slot < cnt) dgt = (s_key[it[j]] >> shift) & (RB_DIGITS - 1);
            dig[j] = (uint8_t)dgt;
            const uint32_t r = s_cnt[dgt * RB_THREADS + tid];
            rk[j] = (uint8_t)r;
            s_cnt[dgt * RB_THREADS + tid] = r + 1;
        }
        __syncthreads();
        // exclusive scan over (digit, thread) in digit-major order
        uint32_t v[RB_DIGITS];
        uint32_t sum = 0;
#pragma unroll
        for (int j = 0; j < RB_DIGITS; ++j) {
            v[j] = s_cnt[tid * RB_DIGITS + j];
            sum += v[j];
        }
        uint32_t tot;
        uint32_t base = block_excl_scan(sum, s_wsum, &tot);
#pragma unroll
        for (int j = 0; j < RB_DIGITS; ++j) {
            s_cnt[tid * RB_DIGITS + j] = base;
            base += v[j];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < RB_IPT; ++j) {
            const uint32_t pos = s_cnt[dig[j] * RB_THREADS + tid] + rk[j];
            s_item[cur ^ 1][pos] = it[j];
        }
        __syncthreads();
        cur ^= 1;
    }

    // runs of equal key in sorted order
    uint32_t head[RB_IPT];
    uint32_t nh = 0;
#pragma unroll
    for (int j = 0; j < RB_IPT; ++j) {
        const int slot = tid * RB_IPT + j;
        uint32_t h = 0;
        if (slot < cnt) {
            const uint32_t k = s_key[s_item[cur][slot]];
            h = (slot == 0) || (k != s_key[s_item[cur][slot - 1]]);
        }
        head[j] = h;
        nh += h;
    }
    uint32_t n_runs;
    uint32_t rbase = block_excl_scan(nh, s_wsum, &n_runs);
    // run start positions into s_cnt (reused), then counts
    uint32_t r = rbase;
#pragma unroll
    for (int j = 0; j < RB_IPT; ++j)
        if (head[j]) s_cnt[r++] = (uint32_t)(tid * RB_IPT + j);
    if (tid == 0) s_cnt[n_runs] = (uint32_t)cnt;
    __syncthreads();
    const int64_t rt = tile * RB_TILE;
    for (uint32_t q = tid; q < n_runs; q += RB_THREADS) {
        const uint32_t st = s_cnt[q], len = s_cnt[q + 1] - st;
        const uint32_t key = s_key[s_item[cur][st]] + kmin;
        sc.run_key[rt + q] = key;
        sc.run_info[rt + q] = st | (len << 16);
        atomicAdd(&sc.key_cnt[key], len);
        atomicAdd(&sc.key_nruns[key], 1u);
    }
    for (int i = tid; i < cnt; i += RB_THREADS) sc.perm[rt + i] = s_item[cur][i];
    if (tid == 0) sc.tile_nruns[tile] = n_runs;
}

// Pass 2: single-pass scan (decoupled look-back) of the per-key (count, runs)
// pairs.  Each 64-bit state word holds flag << 62 | count << 31 | runs.
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
            __hip_atomic_store(&sc.scan_state[0], ST_PRE | agg, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(&sc.scan_state[bid], ST_AGG | agg, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            int64_t j = (int64_t)bid - 1;
            uint32_t spins = 0;
            while (j >= 0) {
                const uint64_t st = __hip_atomic_load(&sc.scan_state[j], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
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
            __hip_atomic_store(&sc.scan_state[bid], ST_PRE | incl, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
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
__global__ __launch_bounds__(256) void k_rebin_lists(RebinScratch sc) {
    const int64_t tile = blockIdx.x;
    const uint32_t nr = sc.tile_nruns[tile];
    for (uint32_t q = threadIdx.x; q < nr; q += blockDim.x) {
        const uint32_t a = (uint32_t)(tile * RB_TILE + q);
        const uint32_t key = sc.run_key[a];
        const uint32_t slot = sc.list_off[key] + atomicAdd(&sc.key_fill[key], 1u);
        sc.list[slot] = a;
    }
}

// Pass 3b: a run's place among the runs of its key is the particle count of
// the runs of that key in earlier tiles (lower run address).
__global__ __launch_bounds__(256) void k_rebin_place(RebinScratch sc) {
    const int64_t tile = blockIdx.x;
    const uint32_t nr = sc.tile_nruns[tile];
    for (uint32_t q = threadIdx.x; q < nr; q += blockDim.x) {
        const uint32_t a = (uint32_t)(tile * RB_TILE + q);
        const uint32_t key = sc.run_key[a];
        const uint32_t l0 = sc.list_off[key], l1 = sc.list_off[key + 1];
        uint32_t before = 0;
        for (uint32_t j = l0; j < l1; ++j) {
            const uint32_t b = sc.list[j];
            if (b < a) before += sc.run_info[b] >> 16;
        }
        sc.run_dest[a] = sc.key_base[key] + before;
    }
}

// Pass 4: LDS-staged scatter.  Thread t handles sorted slots t + 256 i, so a
// wavefront writes 64 consecutive slots, which are consecutive destinations
// inside a run.
__global__ __launch_bounds__(RB_THREADS) void k_rebin_scatter(int64_t n, RebinScratch sc, Cols cols,
                                                             uint32_t *status) {
    __shared__ uint16_t s_rstart[RB_TILE + 1];
    __shared__ uint32_t s_rdest[RB_TILE];
    __shared__ uint64_t s_stage[RB_TILE];
    const int tid = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const int64_t lo = tile * RB_TILE;
    const int cnt = (int)min((int64_t)RB_TILE, n - lo);
    const uint32_t nr = sc.tile_nruns[tile];
    for (uint32_t q = tid; q < nr; q += RB_THREADS) {
        s_rstart[q] = (uint16_t)(sc.run_info[lo + q] & 0xffffu);
        s_rdest[q] = sc.run_dest[lo + q];
    }
    if (tid == 0) s_rstart[nr] = (uint16_t)min(cnt, 0xffff);
    __syncthreads();
    uint32_t dst[RB_IPT];
    uint16_t src[RB_IPT];
#pragma unroll
    for (int i = 0; i < RB_IPT; ++i) {
        const int j = tid + i * RB_THREADS;
        dst[i] = 0;
        src[i] = 0;
        if (j < cnt) {
            src[i] = sc.perm[lo + j];
            // run holding slot j: last run start <= j
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
    for (int c = 0; c < cols.n; ++c) {
        if (cols.bytes[c] == 8) {
            const uint64_t *in = (const uint64_t *)cols.in[c] + lo;
            uint64_t *out = (uint64_t *)cols.out[c];
#pragma unroll
            for (int i = 0; i < RB_IPT; ++i) {
                const int j = tid + i * RB_THREADS;
                if (j < cnt) s_stage[j] = in[j];
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < RB_IPT; ++i) {
                const int j = tid + i * RB_THREADS;
                if (j < cnt && dst[i] != 0xffffffffu) out[dst[i]] = s_stage[src[i]];
            }
        } else {
            const uint32_t *in = (const uint32_t *)cols.in[c] + lo;
            uint32_t *out = (uint32_t *)cols.out[c];
            uint32_t *st = (uint32_t *)s_stage;
#pragma unroll
            for (int i = 0; i < RB_IPT; ++i) {
                const int j = tid + i * RB_THREADS;
                if (j < cnt) st[j] = in[j];
            }
            __syncthreads();
#pragma unroll
            for (int i = 0; i < RB_IPT; ++i) {
                const int j = tid + i * RB_THREADS;
                if (j < cnt && dst[i] != 0xffffffffu) out[dst[i]] = st[src[i]];
            }
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------- deposit

template <int N>
__device__ __forceinline__ void wave_sum(double (&acc)[N]) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
#pragma unroll
        for (int c = 0; c < N; ++c) acc[c] = __dadd_rn(acc[c], __shfl_xor(acc[c], o, 64));
}

// A wavefront per bin: PIT sums weights per leaf corner, PIDT per stencil slot
// of the owning vertex.  With per-particle charges the terms are q_p w_c,
// otherwise w_c (the uniform charge is applied per vertex).
template <int D, int SCHEME, bool REG>
__global__ __launch_bounds__(256) void k_deposit_bins(DevTree t, DevInst in0, F64Ptrs P, int64_t n,
                                                      const int64_t *bin_start, int64_t n_bins, const double *q,
                                                      double *partial) {
    constexpr int NS = SCHEME == PIC_PIT ? (1 << D) : (D == 2 ? 9 : 27);
    const int lane = threadIdx.x & 63;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t b = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); b < n_bins; b += waves) {
        int ii = 0;
        if (t.n_inst > 1) ii = SCHEME == PIC_PIT ? t.leaf_inst[b] : t.pidt_inst[b];
        const DevInst &in = t.n_inst > 1 ? t.inst[ii] : in0;
        const int lev = REG ? in.L : (SCHEME == PIC_PIT ? t.leaf_level[b] : t.pidt_level[b]);
        const int e = in.L - lev;
        const double s = (double)pow3_u32(e);
        const uint32_t su = pow3_u32(e);
        const double rinv = in.rinv[lev];
        double acc[NS];
#pragma unroll
        for (int c = 0; c < NS; ++c) acc[c] = 0.0;
        int64_t p0 = bin_start[b], p1 = bin_start[b + 1];
        if (p0 < 0 || p1 > n || p0 > p1) {             // malformed offsets: flag, touch nothing
            if (lane == 0) flag_status(t.status, PIC_DEV_RANGE);
            p0 = p1 = 0;
        }
        for (int64_t p = p0 + lane; p < p1; p += 64) {
            uint32_t bad = 0;
            Axis ax[D];
            uint32_t a[D];
            double f[D], g[D];
#pragma unroll
            for (int k = 0; k < D; ++k) {
                ax[k] = scale_axis(P.x[k][p], in.Sd, in.S, bad);
                const uint32_t I = ax[k].T >> 1;
                a[k] = REG ? I : div_pow3(I, e);
                f[k] = __dmul_rn(__dsub_rn(ax[k].y, (double)a[k] * s), rinv);
                g[k] = __dsub_rn(1.0, f[k]);
            }
            const double qp = q ? q[p] : 1.0;
            if (SCHEME == PIC_PIT) {
#pragma unroll
                for (int c = 0; c < (1 << D); ++c) {
                    double wc = (c & 1) ? f[0] : g[0];
#pragma unroll
                    for (int k = 1; k < D; ++k) wc = __dmul_rn(wc, ((c >> k) & 1) ? f[k] : g[k]);
                    acc[c] = __dadd_rn(acc[c], q ? __dmul_rn(qp, wc) : wc);
                }
            } else {
                // The owner is the corner nearest to the particle.  Per axis the
                // particle's two corner weights (g, f) land on stencil offsets
                // {0,+1} (owner below) or {-1,0} (owner above); the 3^d slot
                // weights are the tensor product of these per-axis triples, so
                // every slot is updated branch-free (absent ones with +0).
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
                    acc[sl] = __dadd_rn(acc[sl], q ? __dmul_rn(qp, wc) : wc);
                }
            }
        }
        wave_sum<NS>(acc);
        if (lane == 0) {
#pragma unroll
            for (int c = 0; c < NS; ++c) partial[b * NS + c] = acc[c];
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
                    const int64_t leaf = in.leaf_off + peano_low<D>(cell, in.L);
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
                    const int64_t bin = in.pidt_off + peano_low<D>(sh, in.L);
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
    const bool reg = t->all_regular;
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
    const bool reg = t->all_regular;
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
    size_t perm, run_key, run_info, run_dest, tile_nruns, key_cnt, key_nruns, key_fill, key_base, list_off,
        list, scan_state, scan_ctr, total;
};

static RebinLayout rebin_layout(int64_t n, int64_t n_bins) {
    RebinLayout L{};
    const int64_t tiles = (n + RB_TILE - 1) / RB_TILE;
    const int64_t slots = tiles * RB_TILE;
    const int64_t keys = 2 * n_bins;
    const int64_t scan_blocks = (keys + SCAN_TILE - 1) / SCAN_TILE;
    size_t o = 0;
    L.perm = o; o = align256(o + slots * 2);
    L.run_key = o; o = align256(o + slots * 4);
    L.run_info = o; o = align256(o + slots * 4);
    L.run_dest = o; o = align256(o + slots * 4);
    L.tile_nruns = o; o = align256(o + tiles * 4);
    L.key_cnt = o; o = align256(o + keys * 4);      // key_cnt, key_nruns, key_fill contiguous:
    L.key_nruns = o; o = align256(o + keys * 4);    // one fill clears all three
    L.key_fill = o; o = align256(o + keys * 4);
    L.scan_state = o; o = align256(o + scan_blocks * 8);
    L.scan_ctr = o; o = align256(o + 4);
    L.key_base = o; o = align256(o + keys * 4);
    L.list_off = o; o = align256(o + (keys + 1) * 4);
    L.list = o; o = align256(o + slots * 4);
    L.total = o;
    return L;
}

size_t rebin_scratch_bytes(const pic_tree *t, int64_t n, int scheme) {
    return rebin_layout(n, n_bins_of(t, scheme)).total;
}

hipError_t launch_rebin(const pic_tree *t, int scheme, int64_t n, const uint32_t *new_bin, const int64_t *old_start,
                        const Cols &cols, int64_t *new_start, void *scratch, size_t scratch_bytes, hipStream_t s) {
    const int64_t n_bins = n_bins_of(t, scheme);
    const RebinLayout L = rebin_layout(n, n_bins);
    if (scratch_bytes < L.total) return hipErrorInvalidValue;
    char *base = (char *)scratch;
    RebinScratch sc;
    sc.perm = (uint16_t *)(base + L.perm);
    sc.run_key = (uint32_t *)(base + L.run_key);
    sc.run_info = (uint32_t *)(base + L.run_info);
    sc.run_dest = (uint32_t *)(base + L.run_dest);
    sc.tile_nruns = (uint32_t *)(base + L.tile_nruns);
    sc.key_cnt = (uint32_t *)(base + L.key_cnt);
    sc.key_nruns = (uint32_t *)(base + L.key_nruns);
    sc.key_fill = (uint32_t *)(base + L.key_fill);
    sc.key_base = (uint32_t *)(base + L.key_base);
    sc.list_off = (uint32_t *)(base + L.list_off);
    sc.list = (uint32_t *)(base + L.list);
    sc.scan_state = (uint64_t *)(base + L.scan_state);
    sc.scan_ctr = (uint32_t *)(base + L.scan_ctr);
    const int64_t keys = 2 * n_bins;
    const int64_t tiles = (n + RB_TILE - 1) / RB_TILE;
    // counters, scan flags and the block counter start at zero (fill kernel,
    // not a memset node, so the sequence can be captured in a graph)
    const int64_t zero_words = (int64_t)((L.key_base - L.key_cnt) / 4);
    PIC_LAUNCH("rebin_clear", k_fill_u32, dim3(grid_for(zero_words, 256, 4096)), dim3(256), 0, s,
                       (uint32_t *)(base + L.key_cnt), zero_words, 0u);
    if (n > 0)
        PIC_LAUNCH("rebin_tiles", k_rebin_tiles, dim3(tiles), dim3(RB_THREADS), 0, s, new_bin, old_start, n,
                           (uint32_t)n_bins, sc, t->dt.status);
    const int64_t scan_blocks = (keys + SCAN_TILE - 1) / SCAN_TILE;
    PIC_LAUNCH("rebin_scan", k_rebin_scan, dim3(scan_blocks), dim3(256), 0, s, (uint32_t)keys, (uint32_t)n_bins, n, sc,
                       new_start, t->dt.status);
    if (n > 0) {
        PIC_LAUNCH("rebin_lists", k_rebin_lists, dim3(tiles), dim3(256), 0, s, sc);
        PIC_LAUNCH("rebin_place", k_rebin_place, dim3(tiles), dim3(256), 0, s, sc);
        PIC_LAUNCH("rebin_scatter", k_rebin_scatter, dim3(tiles), dim3(RB_THREADS), 0, s, n, sc, cols, t->dt.status);
    }
    return hipGetLastError();
}

size_t deposit_scratch_bytes(const pic_tree *t, int scheme) {
    const int ns = scheme == PIC_PIT ? (1 << t->dim) : (t->dim == 2 ? 9 : 27);
    return align256((size_t)n_bins_of(t, scheme) * ns * sizeof(double));
}

#define PIC_DISPATCH_DEP(D, SCH, REG)                                                                         \
    do {                                                                                                     \
        PIC_LAUNCH("deposit_bins", (k_deposit_bins<D, SCH, REG>), dim3(grid_for(n_bins, 4, 1 << 18)), dim3(256), 0, s, \
                           t->dt, t->inst0, P, p->n, bin_start, n_bins, q, partial);                               \
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
    const bool reg = t->all_regular;
    if (t->dim == 2) {
        if (scheme == PIC_PIT) { if (reg) PIC_DISPATCH_DEP(2, 0, true); else PIC_DISPATCH_DEP(2, 0, false); }
        else { if (reg) PIC_DISPATCH_DEP(2, 1, true); else PIC_DISPATCH_DEP(2, 1, false); }
    } else {
        if (scheme == PIC_PIT) { if (reg) PIC_DISPATCH_DEP(3, 0, true); else PIC_DISPATCH_DEP(3, 0, false); }
        else { if (reg) PIC_DISPATCH_DEP(3, 1, true); else PIC_DISPATCH_DEP(3, 1, false); }
    }
    return hipGetLastError();
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
