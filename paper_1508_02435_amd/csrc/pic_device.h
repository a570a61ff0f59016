// pic_device.h -- device helpers shared by the kernel sources: exact
// division by powers of 3, scaled coordinates, the Peano rank and the tree
// descent, the FP64 gather + push of one particle (push_one), block scans,
// the scratch layout of the re-bin and the fused step, and the fixed-order
// lane reductions of the deposit.
#pragma once

#include <hip/hip_runtime.h>

#include "pic_host.h"

namespace pic {

// ------------------------------------------------------------------ helpers

static __constant__ DivMagic c_magic[PIC_MAX_LEVEL + 2] = {
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

// Scalar passes of the field gather.  PIT: two (a wavefront of one bin
// covers one or two cells).  PIDT: one; a bin spans the 2^d cells around
// its vertex, and further serial passes cost more than the per-lane gathers
// they replace (measured on the 2D and 3D plasma).
template <int D, int SCHEME>
constexpr int field_passes() {
    return SCHEME == PIC_PIT ? 2 : 1;
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
    // wavefront mostly share a few cells: up to field_passes passes serve the
    // lanes whose cell is that of the first pending lane (the id of corner 0
    // names the cell) with scalar loads, and only the lanes left gather per
    // lane.  The values, and so the arithmetic, are the same either way.
    double Ec[D == 2 ? 4 : 1][D];   // 2D: the corner values; 3D: the interpolant ef instead
    double ef[D];
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

// One axis of a free-streaming move: x + v dt, then the wall rule.  Periodic:
// x - floor(x), 1 -> 0 (the push's wrap).  Reflecting: mirrored at 0 (x ->
// -x) or at 1 (x -> 2 - x, exact for x in [1, 2)), with the velocity
// component negated; a landing exactly on 1 goes to the largest double below
// 1.  A move that one mirror cannot bring back into the box is flagged and
// clamped (the bin stays in range).
template <int BC>
__device__ __forceinline__ void stream_axis(double &x, double &v, double dt, uint32_t &bad) {
    double y = __dadd_rn(x, __dmul_rn(v, dt));
    if (BC == PIC_PERIODIC) {
        y = __dsub_rn(y, floor(y));
        if (y == 1.0) y = 0.0;
    } else if (y < 0.0) {
        y = -y;
        v = -v;
    } else if (y >= 1.0) {
        y = __dsub_rn(2.0, y);
        v = -v;
        if (y == 1.0) y = 0x1.fffffffffffffp-1;
    }
    if (!(y >= 0.0 && y < 1.0)) {
        bad |= (y - y == 0.0) ? PIC_DEV_RANGE : PIC_DEV_NONFINITE;
        y = (y >= 1.0) ? 0x1.fffffffffffffp-1 : 0.0;
    }
    x = y;
}

// A free-streaming move of one particle (the particle-handling benchmark):
// stream_axis per axis, then `flops` artificial operations (a dependent
// multiply-add chain whose result only feeds a test that never holds); with
// KEY the particle's new bin (the bin locate gives).
template <int D, int SCHEME, bool REG, int BC, bool KEY>
__device__ __forceinline__ uint32_t stream_one(const DevTree &t, const DevInst &in, const int32_t *lds, int lds_n,
                                               double (&xv)[D], double (&vv)[D], double dt, int flops,
                                               uint32_t &bad) {
#pragma unroll
    for (int k = 0; k < D; ++k) stream_axis<BC>(xv[k], vv[k], dt, bad);
    if (flops > 0) {
        // unrolled: one taken branch per sixteen operations instead of per
        // two, so a wave waits on the chain's own latency and a few resident
        // waves keep the VALU busy
        double a = xv[0];
        const int pairs = flops / 2;
#pragma unroll 8
        for (int f = 0; f < pairs; ++f) a = __dadd_rn(__dmul_rn(a, 0.5), 0.25);
        if (a < -1.0) bad |= PIC_DEV_RANGE;
    }
    if (!KEY) return 0u;
    Axis ax[D];
#pragma unroll
    for (int k = 0; k < D; ++k) ax[k] = scale_axis(xv[k], in.Sd, in.S, bad);
    return bin_of<D, SCHEME, REG>(t, in, ax, lds, lds_n);
}

// How the fused step moves a particle: the leapfrog push of the PIC step, or
// free streaming with periodic or reflecting walls (the particle-handling
// benchmark, no field).  MOVE_STORED is the writing pass's form when the key
// pass has stored the moved state: it only moves records.
constexpr int MOVE_PUSH = 0, MOVE_STREAM_PERIODIC = 1, MOVE_STREAM_REFLECTING = 2, MOVE_STORED = 3;
static_assert(MOVE_STREAM_PERIODIC - 1 == PIC_PERIODIC && MOVE_STREAM_REFLECTING - 1 == PIC_REFLECTING,
              "a streaming move's wall rule is MOVE - 1");

// Key of one particle of the fused step: pushes it (push_one, so the same
// state and bin as every other pass) and returns 2 * new bin + arrived.  A
// particle stays iff its slot lies in its new bin's old segment.  When the
// slot lies in the old segment of the bin of its old cell, that is the case
// iff the two bins agree; the lanes of a wavefront mostly share that cell, so
// its bin and segment come from scalar loads.  Other lanes load the new bin's
// segment.  Call with every lane of the wavefront that holds a particle.
// xv, vv: the particle's state, loaded by the caller (and pushed here).
template <int D, int SCHEME, bool REG, bool MULTI, int MOVE = MOVE_PUSH>
__device__ __forceinline__ uint32_t step_key_one(const DevTree &t, const DevInst &in0, const F64Ptrs &P, int64_t p,
                                                 double (&xv)[D], double (&vv)[D], double qmdt0, double dt0,
                                                 const double *qa, const double *da, const int64_t *inst_start,
                                                 const int64_t *old_start, uint32_t n_bins, const int32_t *lds,
                                                 int lds_n, uint32_t &bad, int flops = 0) {
    int ii = 0;
    if (MULTI) ii = inst_of(inst_start, t.n_inst, p);
    const DevInst &in = MULTI ? t.inst[ii] : in0;
    const double qmdt = (MULTI && qa) ? qa[ii] : qmdt0;
    const double dt = (MULTI && da) ? da[ii] : dt0;
    // lattice index of the old position's bin on a regular instance: its
    // finest cell (PIT) or its nearest vertex on the shifted lattice (PIDT),
    // as bin_of forms them (clamped: it is only a hint, checked below).  Not
    // for 3D PIDT, where the registers it holds cost more than it saves.
    constexpr bool HINT = REG && (SCHEME == PIC_PIT || D == 2);
    uint32_t cold = 0;
    if (HINT) {
        const uint32_t S = (uint32_t)in.S;
        uint32_t m = 1;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const double y = x_scaled(xv[k], in.Sd);
            uint32_t c;
            if (SCHEME == PIC_PIT) {
                c = min((uint32_t)max(y, 0.0), S - 1u);
            } else {
                const uint32_t T = (uint32_t)fmin(fmax(floor(2.0 * y), 0.0), (double)(2u * S - 1u));
                c = (T + 1u) >> 1;
                if (c >= S) c -= S;
                c += (S - 1u) >> 1;
                if (c >= S) c -= S;
            }
            cold += __umul24(c, m);
            m = __umul24(m, S);
        }
    }
    uint32_t b;
    if constexpr (MOVE == MOVE_PUSH)
        b = push_one<D, SCHEME, REG, false>(t, in, P, lds, lds_n, xv, vv, qmdt, dt, p, bad);
    else
        b = stream_one<D, SCHEME, REG, MOVE - 1, true>(t, in, lds, lds_n, xv, vv, dt, flops, bad);
    if (b >= n_bins) bad |= PIC_DEV_RANGE;
    b = min(b, n_bins - 1);
    bool stay = false, known = !old_start;
    if (HINT && !MULTI && old_start) {
        uint64_t pend = __ballot(1);
        const uint32_t off = (uint32_t)(SCHEME == PIC_PIT ? in.leaf_off : in.pidt_off);
#pragma unroll
        for (int it = 0; it < 2; ++it) {
            if (!pend) break;
            const uint32_t cu = (uint32_t)__builtin_amdgcn_readlane((int)cold, __builtin_ctzll(pend));
            const bool mine = cold == cu;
            pend &= ~__ballot(mine);
            const uint32_t ob = off + ld_const(t.peano_tab, (uint32_t)in.ptab + cu);
            const int64_t s0 = ld_const(old_start, ob), s1 = ld_const(old_start, ob + 1u);
            if (mine && s0 <= p && p < s1) {
                stay = b == ob;
                known = true;
            }
        }
    }
    if (!known) stay = old_start[b] <= p && p < old_start[b + 1];
    return 2u * b + (stay ? 0u : 1u);
}

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
constexpr int KLIST_CAP = 128;  // most runs per key listed directly by the fused step's ranking
constexpr int RB_MAX_TILE = 4096;

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
    uint32_t *klist;      // 2*n_bins * klist_cap: fused step, run addresses per key (arrival order)
    uint32_t *khead;      // 2*n_bins (zeroed per call): runs of a key past klist_cap, a linked list
    uint32_t *knext;      // n_tiles * TILE: next run of that list (run address + 1; 0 ends it)
    uint32_t *wave_bin;   // n_tiles * TILE / 64: old bin of slot 64 c (sorted input), for the FP32 form
    uint32_t *run_pos;    // n_tiles * TILE: fused step, a run's position among all runs sorted by (key, tile)
    double *run_part;     // fused step with the deposit in the writing pass: per run (by run_pos) its
                          // particles' summed weights, ns doubles
    uint32_t klist_cap;   // runs per key in the direct list (16..KLIST_CAP, from particles per key)
};

// Scan shapes: the three-call re-bin scans SCAN_TILE keys per block, the
// fused step SP_KEYS; state words hold flag << 62 | count << 31 | runs.
constexpr int SCAN_IPT = 8;
constexpr int SCAN_TILE = 256 * SCAN_IPT;
constexpr uint64_t ST_AGG = 1ull << 62, ST_PRE = 2ull << 62, ST_VAL = (1ull << 62) - 1;
constexpr int SP_THREADS = 256;
constexpr int SP_KPT = 4;                       // keys per thread
constexpr int SP_KEYS = SP_THREADS * SP_KPT;

// Pass 3b: a run's place among the runs of its key is the particle count of
// the key's runs from earlier tiles (lower run address).  Each wavefront
// takes four keys, one per 16-lane group; a list of up to 16 runs is sorted by
// address with a bitonic sort inside its group and prefix-summed.  Longer
// lists are then handled by the whole wavefront: up to 64 runs with a 64-lane
// bitonic sort, beyond that by counting the smaller addresses per run.
template <int W>
__device__ __forceinline__ void place_sorted(const RebinScratch &sc, const uint32_t *lst, uint32_t l0, uint32_t len,
                                             uint32_t kb, int sub, uint32_t *pos = nullptr, uint32_t pos0 = 0u) {
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
    if ((uint32_t)sub < len) {
        sc.run_dest[a] = kb + x - c;
        if (pos) pos[a] = pos0 + (uint32_t)sub;   // the run's place among the key's runs
    }
}

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

// The same chunks walked backwards: an XCD starts at the end of its chunk,
// where the previous pass over the same chunks wrote last (still in its L2
// and in the memory-side cache).
__device__ __forceinline__ int64_t xcd_tile_rev(int64_t b, int64_t tiles) {
    const int64_t x = b & 7, k = b >> 3, q = tiles >> 3, r = tiles & 7;
    const int64_t size = q + (x < r ? 1 : 0);
    return x * q + (x < r ? x : r) + (size - 1 - k);
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

}  // namespace pic
