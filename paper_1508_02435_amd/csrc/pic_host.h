// pic_host.h -- host-side objects of the library (not part of the C ABI).
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

#include "../../include/pic.h"
#include "pic_internal.h"

namespace pic {

// One instance, built on the host (forest-local indices).
struct HostInst {
    int L = 0;
    int64_t S = 1;
    int regular = 0;
    std::vector<int32_t> node_child;   // compacted descent table (local indices)
    std::vector<uint32_t> uni_base;    // local leaf rank
    std::vector<uint32_t> uni_meta;
    std::vector<uint64_t> leaf_key;
    std::vector<uint8_t> leaf_level;
    std::vector<uint32_t> leaf_coord;  // n_leaves * dim
    std::vector<int32_t> leaf_vtx;     // local vertex ids
    std::vector<int32_t> leaf_pidt;    // local PIDT bins
    std::vector<int64_t> vtx_lin;      // sorted lexicographic positions
    std::vector<uint64_t> pidt_key;
    std::vector<uint8_t> pidt_level;
    std::vector<uint32_t> pidt_b;      // n_pidt * dim
    std::vector<int32_t> pidt_vtx;
};

pic_status build_instance(int dim, int L, const uint8_t *masks, HostInst &out);
void build_incidence(int dim, const HostInst &h, int32_t leaf_off, int32_t pidt_off,
                     std::vector<std::vector<int32_t>> &vinc_rows,
                     std::vector<std::vector<int32_t>> &vpinc_rows);
uint64_t host_peano(int dim, const uint32_t *a, int nd);

// Launch-shape knobs.  Every tree carries its own set (pic_tree_tune_set),
// copied from the process defaults (pic_tune_set) when the tree is created.
struct Tuning {
    int rebin_ipt = 8;      // particles per thread in a rebin tile: 8 (2048 tile) or 16 (4096 tile)
    int rebin_radix = 4;    // bits per LDS radix pass: 4 or 5
    int scatter_mode = 0;   // 0: LDS-staged scatter, 1: direct gather from the tile
    int scatter_nt = 0;     // 1: non-temporal stores of the re-binned records
    int scatter_group = 4;  // columns a scatter thread holds in registers at once: 1, 2 or 4
    int deposit_lanes = 0;  // lanes per bin in the deposit: 16, 32 or 64; 0 = by dimension (deposit_lanes_of)
    int step_ipt = 0;       // particles per thread in a fused-step tile: 4, 8 or 16 (1024, 2048, 4096 tile);
                            // 0 = by dimension (step_ipt_of)
    int xcd_tiles = 1;      // 1 = tiles dealt to the 8 XCDs in contiguous chunks, 0 = block order
    int emit_threads = 1024; // threads per emit block: 512 or 1024
    int step_fuse = 2;      // fused step: 1 = key pass and tile ranking in one kernel, 0 = two kernels,
                            // 2 = one kernel for 2D regular single trees with PIT
    int key_stores = 2;     // fused step: the key pass stores the pushed state in place and the writing pass
                            // moves it: 1 always, 0 never, 2 for the FP32 form of 3D trees
    int group_match = 0;    // fused step's ranking pass: 1 = by wavefront key matching, 0 = by LDS tags and masks
    int emit_deposit = 2;   // fused step, 2D regular single trees, uniform charge: 1 = the writing pass deposits,
                            // 2 = it does for PIT only
    int deposit_bpw = 1;    // bins a deposit lane group takes one after the other: 1 or 2
    int deposit_batch = 64; // particles a deposit lane group takes per round: 64 or 256
    int regular_tables = 1; // build Peano rank tables for regular instances (read when a tree is created)
};
extern Tuning g_tune;      // process defaults for trees created afterwards
// Knob by name: set returns false for unknown names or values; get returns -1.
bool tune_set(Tuning &t, const char *name, int64_t value);
int64_t tune_get(const Tuning &t, const char *name);

}  // namespace pic

// The opaque tree object of the C ABI.
struct pic_tree {
    int32_t dim = 0, n_inst = 0, all_regular = 1, max_level = 0;
    int32_t reg_kernels = 0;  // every instance regular with a Peano table: arithmetic kernels apply
    std::vector<pic::HostInst> inst;
    std::vector<int64_t> leaf_off, vtx_off, pidt_off, node_off;  // n_inst + 1 each
    std::vector<uint8_t> image;        // host copy of the device image
    int64_t device_bytes = 0;
    // byte offsets of the tables inside the image
    int64_t o_status = 0, o_inst = 0, o_node = 0, o_ubase = 0, o_umeta = 0, o_llev = 0, o_lvtx = 0,
            o_lpidt = 0, o_plev = 0, o_linst = 0, o_pinst = 0, o_vinst = 0, o_vptr = 0, o_vinc = 0,
            o_vpptr = 0, o_vpinc = 0, o_ptab = 0, o_ctab = 0, o_lcoord = 0, o_pb = 0;
    int64_t n_nodes = 0, n_vinc = 0, n_vpinc = 0;
    void *dev = nullptr;               // bound device buffer (caller-owned)
    pic::DevTree dt{};                 // device view, valid once uploaded
    pic::DevInst inst0{};              // instance 0 (passed by value for single trees)
    pic::Tuning tune{};                // launch-shape knobs of this tree
};

namespace pic {

// Particles per thread of the fused step's tiles.  By default 3D trees with
// at most 256 particles per bin on average take 4096-particle tiles: the
// movers of a bin scatter over its 26 neighbours, so with few particles per
// bin the (tile, key) runs are short, and a longer tile holds more of a bin's
// sources (fewer, longer runs: fewer partly written cache lines in the
// writing pass).  Fuller bins already give long runs and every other tree
// takes 2048, which keeps more blocks resident.
// Lanes per bin of the FP64 deposit.  By default 32 for 3D trees (two bins
// per wavefront: on the 3D plasma the per-bin pass takes 0.28 instead of
// 0.34 ms for PIT and 0.66 instead of 0.82 ms for PIDT) and 64 for 2D ones,
// where 32 is slower (adaptive 2D: 0.124 instead of 0.109 ms).
inline int deposit_lanes_of(const pic_tree *t) {
    return t->tune.deposit_lanes ? t->tune.deposit_lanes : (t->dim == 3 ? 32 : 64);
}

inline int step_ipt_of(const pic_tree *t, int64_t n, int64_t n_bins) {
    if (t->tune.step_ipt) return t->tune.step_ipt;
    return t->dim == 3 && n <= 256 * n_bins ? 16 : 8;
}

}  // namespace pic

namespace pic {

// Records HIP events around a kernel launch when profiling is enabled.
class ProfScope {
  public:
    ProfScope(const char *name, hipStream_t s);
    ~ProfScope();

  private:
    const char *name_;
    hipStream_t s_;
    void *a_;
};

// Switches kernel timing off on this thread while it lives (for calls that
// must create no HIP objects).
class ProfSuspend {
  public:
    ProfSuspend();
    ~ProfSuspend();
};

#define PIC_LAUNCH(NAME, KERNEL, GRID, BLOCK, SHMEM, STREAM, ...)                     \
    do {                                                                           \
        ::pic::ProfScope pic_prof_scope_(NAME, STREAM);                            \
        hipLaunchKernelGGL(KERNEL, GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);         \
    } while (0)

// kernel launchers (pic_kernels.hip); all enqueue on `stream`
struct Cols {
    int32_t n;
    const void *in[16];
    void *out[16];
    int32_t bytes[16];
};

hipError_t launch_locate(const pic_tree *t, int scheme, const pic_particles *p, uint32_t *bin,
                         hipStream_t s);
hipError_t launch_gather_push(const pic_tree *t, int scheme, pic_particles *p, const double *const *E,
                              double qmdt, double dt, const pic_push_params *pp, uint32_t *bin,
                              double *Ep, hipStream_t s);
hipError_t launch_rebin(const pic_tree *t, int scheme, int64_t n, const uint32_t *new_bin,
                        const int64_t *old_start, const Cols &cols, int64_t *new_start,
                        void *scratch, size_t scratch_bytes, hipStream_t s);
size_t rebin_scratch_bytes(const pic_tree *t, int64_t n, int scheme);

hipError_t launch_deposit(const pic_tree *t, int scheme, const pic_particles *p,
                          const int64_t *bin_start, const double *q, double q_uniform, double *rho,
                          void *scratch, size_t scratch_bytes, hipStream_t s);
size_t deposit_scratch_bytes(const pic_tree *t, int scheme);
// Address of the library's device-resident deposit scratch on the current
// device (looked up once per device; pic_kernels.hip).
hipError_t noalloc_scratch(void **ptr);
hipError_t launch_status_clear(const pic_tree *t, hipStream_t s);
hipError_t launch_step(const pic_tree *t, int scheme, pic_particles *in, const int64_t *old_start,
                       const double *const *E, double qmdt, double dt, const pic_push_params *pp, const Cols &extra,
                       pic_particles *out, int64_t *new_start, int q_col, double q_uniform, double *rho,
                       void *scratch, size_t scratch_bytes, void *stats, hipStream_t s);
hipError_t launch_gather_push_f32(const pic_tree *t, int scheme, pic_particles *p, const double *const *E,
                                  double qmdt, double dt, const pic_push_params *pp, const int64_t *bin_start,
                                  const uint32_t *tile_bin, int tile, uint32_t *bin, hipStream_t s);
hipError_t launch_deposit_f32(const pic_tree *t, int scheme, const pic_particles *p, const int64_t *bin_start,
                              const double *q, double q_uniform, double *rho, void *scratch, size_t scratch_bytes,
                              hipStream_t s);
hipError_t launch_convert(const pic_tree *t, int scheme, int to_precision, pic_particles *p, double dt,
                          const pic_push_params *pp, const int64_t *bin_start, uint32_t *bin, hipStream_t s);
size_t step_f32_scratch_bytes(const pic_tree *t, int64_t n, int scheme);
hipError_t launch_step_f32(const pic_tree *t, int scheme, pic_particles *in, const int64_t *old_start,
                           const double *const *E, double qmdt, double dt, const pic_push_params *pp,
                           const Cols &extra, pic_particles *out, int64_t *new_start, int q_col, double q_uniform,
                           double *rho, void *scratch, size_t scratch_bytes, void *stats, hipStream_t s);
hipError_t launch_stream_push(int dim, int64_t n, double *const *x, double *const *v, double dt, hipStream_t s);
// The particle-handling benchmark (pic_move.hip).
hipError_t launch_free_stream(const pic_tree *t, int scheme, pic_particles *p, double dt, const double *dt_dev,
                              int boundary, int flops, uint32_t *bin, hipStream_t s);
hipError_t launch_leaf_counts(const pic_tree *t, const pic_particles *p, unsigned long long *count, hipStream_t s);
hipError_t launch_stream_step(const pic_tree *t, int scheme, pic_particles *in, const int64_t *old_start, double dt,
                              int boundary, int flops, const Cols &extra, pic_particles *out, int64_t *new_start,
                              void *scratch, size_t scratch_bytes, void *stats, hipStream_t s);
pic_status adapt_masks(const pic_tree *t, const int64_t *leaf_count, int64_t ppc, int max_level,
                       std::vector<uint8_t> &masks, int &new_L);
hipError_t launch_vmax(const pic_tree *t, int scheme, const pic_particles *p, const int64_t *bin_start, double dt,
                       double *cells, uint8_t *quiet, void *scratch, hipStream_t s);
size_t vmax_scratch_bytes(const pic_tree *t, int scheme);
int64_t vmax_cells(const pic_tree *t);
// Re-bin statistics of a sorted set (old_start) whose new bins are bins[p] >> shift
// (pic_stats.hip); adds to the caller's pic_rebin_stats record.
hipError_t launch_rebin_stats(const pic_tree *t, int scheme, const int64_t *old_start, const uint32_t *bins,
                              int shift, int64_t n, void *stats, hipStream_t s);

}  // namespace pic
