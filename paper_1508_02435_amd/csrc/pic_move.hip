// pic_move.hip -- the particle-handling benchmark of the paper's results
// section (Sec. 6 setup): free streaming with periodic or reflecting walls
// and artificial flops per move, particle counts per leaf, and the
// ppc-driven refinement and coarsening of a tree (host side).
#include <hip/hip_runtime.h>

#include <unordered_map>
#include <vector>

#include "pic_launch.h"

namespace pic {

template <int D, int SCHEME, bool REG, bool MULTI, int BC>
__global__ __launch_bounds__(256) void k_free_stream(DevTree t, DevInst in0, F64Ptrs P, int64_t n, double dt0,
                                                     const double *dt_arr, const int64_t *inst_start, int flops,
                                                     uint32_t *bin_out) {
    __shared__ int32_t lds[REG ? 1 : PIC_LDS_NODES];
    const int lds_n = MULTI ? 0 : stage_nodes<REG>(t, in0, lds);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        int ii = 0;
        if (MULTI) ii = inst_of(inst_start, t.n_inst, p);
        const DevInst &in = MULTI ? t.inst[ii] : in0;
        const double dt = (MULTI && dt_arr) ? dt_arr[ii] : dt0;
        uint32_t bad = 0;
        double xv[D], vv[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            xv[k] = P.x[k][p];
            vv[k] = P.v[k][p];
        }
        const uint32_t b = stream_one<D, SCHEME, REG, BC, true>(t, in, lds, lds_n, xv, vv, dt, flops, bad);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            P.x[k][p] = xv[k];
            P.v[k][p] = vv[k];
        }
        bin_out[p] = b;
        if (bad) flag_status(t.status, bad);
    }
}

__global__ void k_fill_u64(unsigned long long *a, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = 0ull;
}

// Particles per leaf (forest-wide leaf ranks): integer adds, so the counts
// do not depend on the order of the atomics.
template <int D, bool REG, bool MULTI>
__global__ __launch_bounds__(256) void k_leaf_counts(DevTree t, DevInst in0, F64Ptrs P, int64_t n,
                                                     const int64_t *inst_start, unsigned long long *count) {
    __shared__ int32_t lds[REG ? 1 : PIC_LDS_NODES];
    const int lds_n = MULTI ? 0 : stage_nodes<REG>(t, in0, lds);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += stride) {
        const DevInst &in = MULTI ? t.inst[inst_of(inst_start, t.n_inst, p)] : in0;
        uint32_t bad = 0;
        Axis ax[D];
#pragma unroll
        for (int k = 0; k < D; ++k) ax[k] = scale_axis(P.x[k][p], in.Sd, in.S, bad);
        atomicAdd(&count[bin_of<D, PIC_PIT, REG>(t, in, ax, lds, lds_n)], 1ull);
        if (bad) flag_status(t.status, bad);
    }
}

#define PIC_FS(D, SCH, REG, MULTI)                                                                             \
    do {                                                                                                       \
        if (boundary == PIC_PERIODIC)                                                                          \
            PIC_LAUNCH("free_stream", (k_free_stream<D, SCH, REG, MULTI, PIC_PERIODIC>), dim3(grid), dim3(256), 0, \
                       s, t->dt, t->inst0, P, p->n, dt, da, p->inst_start_dev, flops, bin);                    \
        else                                                                                                   \
            PIC_LAUNCH("free_stream", (k_free_stream<D, SCH, REG, MULTI, PIC_REFLECTING>), dim3(grid), dim3(256), \
                       0, s, t->dt, t->inst0, P, p->n, dt, da, p->inst_start_dev, flops, bin);                 \
    } while (0)
#define PIC_FS_RM(D, SCH)                                                                                      \
    do {                                                                                                       \
        if (multi) { if (reg) PIC_FS(D, SCH, true, true); else PIC_FS(D, SCH, false, true); }                  \
        else { if (reg) PIC_FS(D, SCH, true, false); else PIC_FS(D, SCH, false, false); }                      \
    } while (0)

hipError_t launch_free_stream(const pic_tree *t, int scheme, pic_particles *p, double dt, const double *da,
                              int boundary, int flops, uint32_t *bin, hipStream_t s) {
    if (p->n == 0) return hipSuccess;
    F64Ptrs P = make_ptrs(t, p, nullptr, nullptr);
    const int grid = grid_for(p->n, 256, 1 << 20);
    const bool multi = t->n_inst > 1;
    const bool reg = t->reg_kernels != 0;
    if (t->dim == 2) {
        if (scheme == PIC_PIT) PIC_FS_RM(2, 0); else PIC_FS_RM(2, 1);
    } else {
        if (scheme == PIC_PIT) PIC_FS_RM(3, 0); else PIC_FS_RM(3, 1);
    }
    return hipGetLastError();
}
#undef PIC_FS_RM
#undef PIC_FS

hipError_t launch_leaf_counts(const pic_tree *t, const pic_particles *p, unsigned long long *count,
                              hipStream_t s) {
    const int64_t nl = t->leaf_off.back();
    PIC_LAUNCH("fill", k_fill_u64, dim3(grid_for(nl, 256, 1 << 16)), dim3(256), 0, s, count, nl);
    if (p->n == 0) return hipGetLastError();
    F64Ptrs P = make_ptrs(t, p, nullptr, nullptr);
    const int grid = grid_for(p->n, 256, 1 << 20);
    const bool multi = t->n_inst > 1, reg = t->reg_kernels != 0;
#define PIC_LC(D, REG, MULTI)                                                                                  \
    PIC_LAUNCH("leaf_counts", (k_leaf_counts<D, REG, MULTI>), dim3(grid), dim3(256), 0, s, t->dt, t->inst0, P, \
               p->n, p->inst_start_dev, count)
    if (t->dim == 2) {
        if (multi) { if (reg) PIC_LC(2, true, true); else PIC_LC(2, false, true); }
        else { if (reg) PIC_LC(2, true, false); else PIC_LC(2, false, false); }
    } else {
        if (multi) { if (reg) PIC_LC(3, true, true); else PIC_LC(3, false, true); }
        else { if (reg) PIC_LC(3, true, false); else PIC_LC(3, false, false); }
    }
#undef PIC_LC
    return hipGetLastError();
}

// ------------------------------------------------- raPIDT's v_max attribute
//
// Cells are addressed as in the refine masks, levels 0..L back to back,
// (3^l)^d positions per level, lexicographic.  A wavefront per bin takes the
// largest velocity component of the bin's particles; a thread per leaf then
// takes its value (its own bin for PIT, the largest of its corners' dual
// cells for PIDT) up its ancestor chain with atomicMax on the bit patterns
// (non-negative doubles order like their bits, and max does not depend on
// the order of the updates).

// First cell of level l: sum of (3^j)^d for j < l = (3^(dl) - 1) / (3^d - 1).
__host__ __device__ inline int64_t cell_off(int d, int l) {
    int64_t a = 1, b = 1;
    for (int j = 0; j < d * l; ++j) a *= 3;
    for (int j = 0; j < d; ++j) b *= 3;
    return (a - 1) / (b - 1);
}

__global__ __launch_bounds__(256) void k_vmax_bins(const F64Ptrs P, int dim, const int64_t *bin_start, int64_t n_bins,
                                                   double *bval) {
    const int lane = threadIdx.x & 63;
    const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t b = wid; b < n_bins; b += nw) {
        const int64_t p0 = bin_start[b], p1 = bin_start[b + 1];
        double m = 0.0;
        for (int64_t p = p0 + lane; p < p1; p += 64)
            for (int k = 0; k < dim; ++k) m = fmax(m, fabs(P.v[k][p]));
        for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
        if (lane == 0) bval[b] = m;
    }
}

__global__ void k_fill_cells(unsigned long long *v, uint8_t *mark, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        v[i] = 0ull;
        if (mark) mark[i] = 0;
    }
}

template <int D>
__global__ __launch_bounds__(256) void k_vmax_leaves(DevTree t, int scheme, const double *bval, int64_t n_leaves,
                                                     unsigned long long *cells, uint8_t *mark) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n_leaves; r += stride) {
        double val = 0.0;
        if (scheme == PIC_PIT) {
            val = bval[r];
        } else {
            for (int c = 0; c < (1 << D); ++c) val = fmax(val, bval[t.leaf_pidt[r * (1 << D) + c]]);
        }
        const unsigned long long bits = (unsigned long long)__double_as_longlong(val);
        int64_t a[D];
        for (int k = 0; k < D; ++k) a[k] = t.leaf_coord[r * D + k];
        for (int l = t.leaf_level[r]; l >= 0; --l) {
            int64_t n = 1, idx = 0;
            for (int j = 0; j < l; ++j) n *= 3;
            int64_t m = 1;
            for (int k = 0; k < D; ++k) {
                idx += a[k] * m;
                m *= n;
            }
            const int64_t c = cell_off(D, l) + idx;
            atomicMax(&cells[c], bits);
            if (mark) mark[c] = 1;
            for (int k = 0; k < D; ++k) a[k] /= 3;
        }
    }
}

// The predicate v_max(c) dt <= h(c), h = 1 / 3^l (one rounding), for the
// cells the leaves marked as existing.
__global__ void k_vmax_quiet(const double *cells, int d, int L, double dt, uint8_t *mark) {
    const int64_t n = cell_off(d, L + 1);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if (!mark[i]) continue;
        int l = 0;
        while (cell_off(d, l + 1) <= i) ++l;
        double p3 = 1.0;
        for (int j = 0; j < l; ++j) p3 *= 3.0;
        mark[i] = __dmul_rn(cells[i], dt) <= __ddiv_rn(1.0, p3) ? 1 : 0;
    }
}

hipError_t launch_vmax(const pic_tree *t, int scheme, const pic_particles *p, const int64_t *bin_start, double dt,
                       double *cells, uint8_t *quiet, void *scratch, hipStream_t s) {
    const int L = t->inst[0].L, d = t->dim;
    const int64_t nb = n_bins_of(t, scheme), nl = t->leaf_off.back();
    double *bval = (double *)scratch;   // per-bin values
    const int64_t n_cells = cell_off(d, L + 1);
    F64Ptrs P = make_ptrs(t, p, nullptr, nullptr);
    PIC_LAUNCH("fill", k_fill_cells, dim3(grid_for(n_cells, 256, 1 << 16)), dim3(256), 0, s,
               (unsigned long long *)cells, quiet, n_cells);
    if (nb > 0)
        PIC_LAUNCH("vmax_bins", k_vmax_bins, dim3(grid_for(nb, 4, 1 << 16)), dim3(256), 0, s, P, d, bin_start, nb,
                   bval);
    if (d == 2)
        PIC_LAUNCH("vmax_leaves", k_vmax_leaves<2>, dim3(grid_for(nl, 256, 1 << 16)), dim3(256), 0, s, t->dt, scheme,
                   bval, nl, (unsigned long long *)cells, quiet);
    else
        PIC_LAUNCH("vmax_leaves", k_vmax_leaves<3>, dim3(grid_for(nl, 256, 1 << 16)), dim3(256), 0, s, t->dt, scheme,
                   bval, nl, (unsigned long long *)cells, quiet);
    if (quiet)
        PIC_LAUNCH("vmax_quiet", k_vmax_quiet, dim3(grid_for(n_cells, 256, 1 << 16)), dim3(256), 0, s, cells, d, L,
                   dt, quiet);
    return hipGetLastError();
}

size_t vmax_scratch_bytes(const pic_tree *t, int scheme) {
    return align256((size_t)n_bins_of(t, scheme) * sizeof(double));
}

int64_t vmax_cells(const pic_tree *t) { return cell_off(t->dim, t->inst[0].L + 1); }

// ------------------------------------------------------ ppc-driven adaptation
//
// Per level a dense state byte for every cell position (the layout of the
// refine masks): 0 absent, 1 leaf, 2 refined, 3 leaf to refine, 4 refined
// cell to coarsen.  Leaves come from the tree's leaf table (level and
// coordinates per Peano rank); every ancestor of a leaf is refined.

pic_status adapt_masks(const pic_tree *t, const int64_t *leaf_count, int64_t ppc, int max_level,
                       std::vector<uint8_t> &masks, int &new_L) {
    const pic::HostInst &h = t->inst[0];
    const int d = t->dim, L = h.L;
    const int top = std::max(L, std::min(L + 1, max_level));   // deepest level the new tree can reach
    // powers of 3 up to 3^39 < 2^63 (the tree limits keep d * top <= 36)
    int64_t p3[40];
    p3[0] = 1;
    for (int i = 1; i < 40; ++i) p3[i] = p3[i - 1] * 3;
    if (d * top > 39) return PIC_E_ARG;
    // the dense per-level states: refuse more than 16 GiB for the deepest
    if (p3[d * top] > ((int64_t)1 << 34)) return PIC_E_CAPACITY;
    auto lex = [&](int l, const int64_t *a) {
        int64_t r = 0;
        for (int k = d - 1; k >= 0; --k) r = r * p3[l] + a[k];
        return r;
    };
    std::vector<std::vector<uint8_t>> st(top + 1);
    for (int l = 0; l <= top; ++l) st[l].assign((size_t)p3[d * l], 0);
    // per parent of a leaf: (its leaf children, their particles)
    std::unordered_map<int64_t, std::pair<int, int64_t>> kids;
    const int64_t nl = (int64_t)h.leaf_level.size();
    kids.reserve((size_t)(nl / 4 + 16));
    for (int64_t r = 0; r < nl; ++r) {
        const int l = h.leaf_level[r];
        int64_t a[3];
        for (int k = 0; k < d; ++k) a[k] = h.leaf_coord[(size_t)r * d + k];
        const int64_t id = lex(l, a);
        // refine: an overfull leaf above the level cap
        st[l][id] = (l < max_level && leaf_count[r] > ppc) ? 3 : 1;
        if (l >= 2) {
            int64_t b[3];
            for (int k = 0; k < d; ++k) b[k] = a[k] / 3;
            auto &e = kids[lex(l - 1, b) * 32 + (l - 1)];
            e.first += 1;
            e.second += leaf_count[r];
        }
        for (int up = l - 1; up >= 0; --up) {   // every ancestor is refined
            for (int k = 0; k < d; ++k) a[k] /= 3;
            uint8_t &s = st[up][lex(up, a)];
            if (s == 2) break;
            s = 2;
        }
    }
    // coarsen: a refined non-root cell whose 3^d children are all leaves
    // (none of them refined by the rule above) holding at most ppc particles
    // (a child being refined holds more than ppc by itself, so a cell whose
    // children hold at most ppc has none)
    for (const auto &kv : kids) {
        const int l = (int)(kv.first & 31);
        const int64_t id = kv.first >> 5;
        if (kv.second.first == (int)p3[d] && kv.second.second <= ppc && st[l][id] == 2) st[l][id] = 4;
    }
    // the new masks: a cell is refined iff it is reached through refined
    // cells and is refined (2) or to be refined (3)
    std::vector<std::vector<uint8_t>> ref(top + 1);
    std::vector<uint8_t> live(1, 1);
    new_L = 0;
    for (int l = 0; l <= top; ++l) {
        std::vector<uint8_t> m(st[l].size(), 0);
        bool any = false;
        for (size_t i = 0; i < m.size(); ++i)
            if (live[i] && (st[l][i] == 2 || st[l][i] == 3)) {
                m[i] = 1;
                any = true;
            }
        if (!any) break;
        ref[l].swap(m);
        new_L = l + 1;
        if (l + 1 > top) break;
        std::vector<uint8_t> nxt((size_t)p3[d * (l + 1)], 0);
        for (size_t i = 0; i < ref[l].size(); ++i) {
            if (!ref[l][i]) continue;
            int64_t a[3], r = (int64_t)i;
            for (int k = 0; k < d; ++k) {
                a[k] = r % p3[l];
                r /= p3[l];
            }
            for (int c = 0; c < (int)p3[d]; ++c) {
                int64_t b[3], cc = c;
                for (int k = 0; k < d; ++k) {
                    b[k] = 3 * a[k] + cc % 3;
                    cc /= 3;
                }
                nxt[lex(l + 1, b)] = 1;
            }
        }
        live.swap(nxt);
    }
    masks.clear();
    for (int l = 0; l < new_L; ++l) masks.insert(masks.end(), ref[l].begin(), ref[l].end());
    return PIC_OK;
}

}  // namespace pic
