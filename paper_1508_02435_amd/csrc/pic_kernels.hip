// pic_kernels.hip -- gfx950 kernels of the FP64 path outside the re-bin:
//
// gather_push  one thread per particle: locate the leaf holding x (arithmetic
//              for uniform subtrees, a short descent otherwise, its top levels
//              in LDS), d-linear gather of E from the 2^d leaf corners, leapfrog
//              kick and drift, periodic wrap, and the new bin of the particle
//              (PIT leaf rank or PIDT dual-cell rank).  SoA streams, coalesced.
// locate       the bin of every particle of a set.
// deposit      a wavefront per bin reduces its particles' weights per corner
//              (PIT) or per 3^d stencil slot (PIDT) in a fixed order; a second
//              pass sums, per vertex, the slots that touch it in a fixed order.
//              No floating-point atomics.
// stream_push  the stream benchmark of the paper's evaluation.
#include <hip/hip_runtime.h>

#include <mutex>

#include "pic_launch.h"

namespace pic {

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

// ----------------------------------------------------------------- launchers

Tuning g_tune;

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

size_t deposit_scratch_bytes(const pic_tree *t, int scheme) {
    const int ns = scheme == PIC_PIT ? (1 << t->dim) : (t->dim == 2 ? 9 : 27);
    return align256((size_t)n_bins_of(t, scheme) * ns * sizeof(double));
}

#define PIC_DEP_BINS(D, SCH, REG, G)                                                                          \
    do {                                                                                                      \
        if (small_batch)                                                                                       \
            PIC_LAUNCH("deposit_bins", (k_deposit_bins<D, SCH, REG, G, 64 / G, 1>),                            \
                       dim3(grid_for(n_bins, 256 / G, 1 << 18)), dim3(256), 0, s, t->dt, t->inst0, P, p->n,   \
                       bin_start, n_bins, q, partial);                                                        \
        else if (t->tune.deposit_bpw == 2)                                                                     \
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
        if (deposit_lanes_of(t) == 16) PIC_DEP_BINS(D, SCH, REG, 16);                                         \
        else if (deposit_lanes_of(t) == 32) PIC_DEP_BINS(D, SCH, REG, 32);                                    \
        else PIC_DEP_BINS(D, SCH, REG, 64);                                                                  \
        PIC_LAUNCH("deposit_vertices", (k_deposit_vertices<D, SCH, REG>), dim3(grid_for(n_vtx, 256, 1 << 16)), dim3(256), \
                           0, s, t->dt, t->inst0, partial, n_vtx, q ? 1 : 0, q_uniform, rho);                 \
    } while (0)

void launch_deposit_vertices(const pic_tree *t, int scheme, bool reg, const double *partial, bool use_q,
                             double q_uniform, double *rho, hipStream_t s) {
    const int64_t n_vtx = t->vtx_off.back();
    const dim3 g(grid_for(n_vtx, 256, 1 << 16)), b(256);
#define PIC_DV(D, SCH, REG)                                                                                 \
    PIC_LAUNCH("deposit_vertices", (k_deposit_vertices<D, SCH, REG>), g, b, 0, s, t->dt, t->inst0, partial, n_vtx, \
               use_q ? 1 : 0, q_uniform, rho)
    if (t->dim == 2) {
        if (scheme == PIC_PIT) { if (reg) PIC_DV(2, 0, true); else PIC_DV(2, 0, false); }
        else { if (reg) PIC_DV(2, 1, true); else PIC_DV(2, 1, false); }
    } else {
        if (scheme == PIC_PIT) { if (reg) PIC_DV(3, 0, true); else PIC_DV(3, 0, false); }
        else { if (reg) PIC_DV(3, 1, true); else PIC_DV(3, 1, false); }
    }
#undef PIC_DV
}

hipError_t launch_deposit(const pic_tree *t, int scheme, const pic_particles *p, const int64_t *bin_start,
                          const double *q, double q_uniform, double *rho, void *scratch, size_t scratch_bytes,
                          hipStream_t s) {
    const int64_t n_bins = n_bins_of(t, scheme);
    const int64_t n_vtx = t->vtx_off.back();
    if (scratch_bytes < deposit_scratch_bytes(t, scheme)) return hipErrorInvalidValue;
    double *partial = (double *)scratch;
    F64Ptrs P = make_ptrs(t, p, nullptr, nullptr);
    const bool reg = t->reg_kernels != 0;
    // particles a bin's lane group takes per round: 64 (fewer registers, the
    // default) or 256 (more loads in flight for large bins)
    const bool small_batch = t->tune.deposit_batch == 64;
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

// ------------------------------------------------- deposit without allocation
//
// pic_deposit_noalloc keeps the deposit's per-bin partials in this
// device-resident array instead of a caller buffer.  Each GPU the library
// runs on holds its own copy until the process ends.  In host code the
// array's name stands for a host-side shadow, so the device address is
// looked up once per device (with that device current) and only that
// address is ever handed to kernels.
static __device__ __align__(256) unsigned char noalloc_partials[PIC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(void **ptr) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_partials));
        if (e != hipSuccess) return e;
        g_noalloc_ptr[dev] = p;
    }
    *ptr = g_noalloc_ptr[dev];
    return hipSuccess;
}

}  // namespace pic
