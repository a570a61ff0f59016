/*
 * pic.h -- C ABI of the MI355X spacetree particle-in-cell hot path.
 *
 * One time step of the particle side of a particle-in-cell (PIC) cycle on a
 * k = 3 spacetree (paper "Two Particle-in-Grid Realisations on Spacetrees",
 * Sec. 3 for the cycle, Sec. 4 for the tree, Sec. 5 for the particle
 * stores), split into three calls that run on one GPU stream:
 *
 *   pic_gather_push  field gather E_i = R^T(x_i) E and leapfrog push, and the
 *                    new bin of every particle (leaf for PIT, dual cell for
 *                    PIDT);
 *   pic_rebin        stable reorder of the particle arrays into their new
 *                    bins (Theorems 1 and 2: afterwards every particle is
 *                    stored in the leaf / dual cell that covers it);
 *   pic_deposit      charge deposit rho = sum_i R(x_i) on the vertices.
 *
 * Conventions shared by every call:
 *  - Pointers named *_dev are device pointers, owned by the caller, which
 *    must keep them alive until the stream has finished the call.  Other
 *    pointers are host pointers, read during the call only.
 *  - `stream` is a hipStream_t passed as void*.  Every call only enqueues
 *    work on it (no host synchronisation) unless stated otherwise; results
 *    are deterministic: the same inputs give bit-identical outputs.
 *  - The library allocates no device memory.  Tree tables live in a caller
 *    buffer (pic_tree_upload); temporary storage is a caller scratch buffer
 *    of pic_scratch_bytes() bytes.
 *  - Errors: calls return pic_status; nothing throws or aborts.  Argument
 *    errors are detected on the host before anything is enqueued.  Data
 *    errors found on the device (non-finite or out-of-box coordinates) set a
 *    sticky bit in a status word kept in the tree buffer; every kernel keeps
 *    its indices in range regardless, so the stream stays valid, and
 *    pic_status_sync() reports and clears the word.
 *  - Positions are in the periodic unit box [0,1)^d.  Particle bins are
 *    uint32 ranks in ascending space-filling-curve key order (see
 *    pic_tree_leaf_table); segment offsets `bin_start` are int64.
 *  - Particle counts must stay below 2^31 per call.
 */
#ifndef PIC_H
#define PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pic_status;
#define PIC_OK 0
#define PIC_E_ARG 1        /* bad argument: null pointer, size, enum value */
#define PIC_E_SCRATCH 2    /* scratch buffer smaller than pic_scratch_bytes() */
#define PIC_E_CAPACITY 3   /* an output or tree buffer is too small */
#define PIC_E_NONFINITE 4  /* device: a position or velocity was NaN/Inf */
#define PIC_E_TREE 5       /* malformed tree description */
#define PIC_E_HIP 6        /* a HIP runtime call failed */
#define PIC_E_RANGE 7      /* device: a position lay outside [0,1), or a bin outside the tree */
#define PIC_E_STATE 8      /* call order violated (e.g. tree not uploaded) */
#define PIC_E_MEMORY 9     /* host memory for a builder's tables could not be allocated */

/* Particle storage schemes (paper Sec. 5.1 and Sec. 5.2). */
#define PIC_PIT 0          /* particle in tree: bin = leaf covering x (Theorem 1) */
#define PIC_PIDT 1         /* particle in dual tree: bin = vertex of that leaf whose
                              dual cell covers x (Theorem 2) */

/* Arithmetic forms. */
#define PIC_F64 0          /* x, v in FP64 domain units */
#define PIC_F32_OFFSET 1   /* FP32 offsets within the leaf, FP32 velocity in cells/step */

/* Walls of the unit box for free streaming (pic_free_stream). */
#define PIC_PERIODIC 0     /* x wraps into [0,1) as in the push */
#define PIC_REFLECTING 1   /* x is mirrored at the wall, that velocity component negated */

typedef struct pic_tree pic_tree;   /* opaque host object */

/* ------------------------------------------------------------------ tree */

/*
 * Build the host description of a forest of `n_inst` spacetrees of the same
 * dimension over the periodic unit box (paper Sec. 4: root = unit box, a
 * refined cell has 3^d children, leaves are unrefined cells; Sec. 4.1 dual
 * grid).  A single tree is a forest of one.
 *
 *   dim        2 or 3.
 *   max_level  host, n_inst entries: deepest level L_i of instance i
 *              (0 <= L_i, dim*L_i <= 36).
 *   masks      host: for each instance in turn, for each level l < L_i, a
 *              uint8 array of (3^l)^dim flags in lexicographic order (axis
 *              0 fastest); 1 = the level-l cell is refined.  Flags of cells
 *              whose parent is unrefined are ignored.
 *   out        receives the new object (free with pic_tree_destroy).
 *
 * Errors: PIC_E_ARG for bad sizes or null pointers, PIC_E_TREE if a forest
 * would exceed 2^31 leaves, vertices or nodes.
 */
pic_status pic_tree_create(int32_t dim, int32_t n_inst, const int32_t *max_level,
                           const uint8_t *masks, pic_tree **out);

void pic_tree_destroy(pic_tree *tree);

typedef struct {
    int32_t dim, n_inst;
    int32_t regular;          /* 1 if every instance is uniformly refined */
    int32_t max_level;        /* largest L_i */
    int64_t n_leaves;         /* PIT bins over the forest */
    int64_t n_vertices;       /* distinct leaf-corner positions over the forest */
    int64_t n_pidt;           /* PIDT bins over the forest */
    int64_t n_nodes;          /* descent-table nodes */
    int64_t device_bytes;     /* size of the buffer pic_tree_upload needs */
} pic_tree_info;

pic_status pic_tree_get_info(const pic_tree *tree, pic_tree_info *info);

typedef struct {
    int32_t max_level;        /* L_i */
    int32_t regular;
    int64_t leaf_offset, n_leaves;     /* forest-wide leaf ranks of this instance */
    int64_t vertex_offset, n_vertices; /* forest-wide vertex ids */
    int64_t pidt_offset, n_pidt;       /* forest-wide PIDT ranks */
} pic_instance_info;

pic_status pic_tree_get_instance(const pic_tree *tree, int32_t inst, pic_instance_info *info);

/*
 * Host copies of the tables, for checking and for building fields.  Every
 * output pointer may be NULL.  Sizes: n_leaves (key, level), n_leaves*dim
 * (coord), n_leaves*2^dim (vtx, pidt), n_vertices*dim (pos), n_pidt
 * (pidt_key, pidt_level), n_pidt*dim (pidt_b).
 *   key    leaf key peano_l(a) * 3^(dim*(L-l)) * 64 + l; leaves are ranked by
 *          ascending key within an instance, instances back to back.
 *   coord  leaf coordinates at the leaf's own level.
 *   vtx    forest-wide vertex id of corner c = sum_k b_k 2^k of each leaf.
 *   pidt   forest-wide PIDT bin of each corner at the leaf's level.
 *   pos    vertex position in finest-cell units of its instance; vertices
 *          are numbered per instance in lexicographic order (axis 0 fastest).
 *   pidt_key  peano_L(J') * 64 + l with J' = (b*s + (3^L-1)/2) mod 3^L.
 *   pidt_b    vertex coordinates at the bin's level.
 */
pic_status pic_tree_leaf_table(const pic_tree *tree, uint64_t *key, int32_t *level,
                               int64_t *coord, int32_t *vtx, int32_t *pidt);
pic_status pic_tree_vertex_table(const pic_tree *tree, int64_t *pos);
pic_status pic_tree_pidt_table(const pic_tree *tree, uint64_t *pidt_key, int32_t *pidt_level,
                               int64_t *pidt_b);

/*
 * Copy the device tables into `buffer_dev` (at least info.device_bytes
 * bytes, 256-byte aligned) and bind them to `tree`.  The buffer also holds
 * the sticky status word, cleared here.  The copy runs on `stream` and the
 * call waits for it (synchronises `stream`) before returning; the host
 * tables stay owned by `tree`.
 */
pic_status pic_tree_upload(pic_tree *tree, void *buffer_dev, size_t bytes, void *stream);

/*
 * Return the sticky device status of `tree` (PIC_OK or the first data error
 * code in the order NONFINITE, RANGE) and clear it.  Synchronises `stream`.
 */
pic_status pic_status_sync(pic_tree *tree, void *stream);

const char *pic_status_string(pic_status s);

/* -------------------------------------------------------------- particles */

/*
 * One particle set in structure-of-arrays form.  FP64 form: x[k], v[k]
 * (k < dim) are n doubles each, x in [0,1) domain units, v in domain units
 * per unit time.  FP32 offset form (trees whose instances are all regular,
 * with Peano rank tables): off[k] in [0,1) is the offset inside the
 * particle's finest cell in cell widths and u[k] the velocity in finest cells
 * per step (v dt 3^L); the cell is implicit in the particle's bin: the leaf
 * for PIT, and for PIDT the owner vertex J with the cell J - 1 where
 * off >= 1/2 and J otherwise, per axis.  Unused pointers may be NULL.
 *
 * inst_start_dev: for a forest, n_inst+1 int64 particle offsets: the
 * particles of instance i are [inst_start[i], inst_start[i+1]), in order.
 * NULL for a single tree.  Particles never change instance.
 *
 * For a set a call writes (the `out` of pic_step and pic_stream_step), n is
 * the capacity of its arrays and must equal the input's n, since a step
 * keeps every particle: any other value is rejected with PIC_E_ARG before
 * anything is enqueued.
 */
typedef struct {
    int64_t n;
    double *x[3];
    double *v[3];
    float *off[3];
    float *u[3];
    const int64_t *inst_start_dev;
} pic_particles;

/* Per-instance push parameters for a forest: qmdt[i] = (q/m) dt and dt[i],
   device arrays of n_inst doubles.  NULL pointers select the scalars. */
typedef struct {
    const double *qmdt_dev;
    const double *dt_dev;
} pic_push_params;

/*
 * Locate: the bin of every particle of an unsorted (or sorted) set.
 * bin_dev receives n uint32 forest-wide bins of `scheme`.  Used to start a
 * run from generated particles; pic_gather_push emits bins itself.
 */
pic_status pic_locate(const pic_tree *tree, int32_t scheme, int32_t precision,
                      const pic_particles *p, const int64_t *bin_start_dev,
                      uint32_t *bin_dev, void *stream);

/*
 * Gather + push (paper Sec. 3 steps 3 and 4; d-linear shape functions).
 * For every particle, in place:
 *   E_p = sum_c w_c(x) E[vtx_c]   over the 2^d corners of the leaf holding x,
 *   v  <- v + qmdt * E_p,  x <- x + v * dt,  x <- x - floor(x) (1.0 -> 0.0),
 * then the particle's new bin under `scheme` is written to bin_dev.
 *   E_dev[k]     device, n_vertices doubles: field component k per vertex.
 *   qmdt, dt     (q/m)*dt and dt for a single tree; ignored per instance
 *                when `params` has device arrays.
 *   bin_start_dev  the current segment offsets of p (n_bins+1 int64); needed
 *                by the FP32 form (its cell is implicit in the bin), NULL is
 *                allowed for FP64.
 *   Ep_dev       optional (NULL): dim*n doubles receiving E_p per particle
 *                (FP64 form only).
 * FP64 arithmetic follows a fixed operation order with no fused multiply-add,
 * so x, v and the bins equal a serial IEEE evaluation of the same formulas.
 * FP32 form: E is still FP64 at the vertices; weights, gather and push are
 * FP32, u <- u + fl32(qmdt dt 3^L) E_p, and the cell moves by the integer
 * floor(off + u) (exact, any distance, periodic) with off keeping the
 * fraction.  PIC_E_ARG for FP32 on trees without the tables.
 */
pic_status pic_gather_push(const pic_tree *tree, int32_t scheme, int32_t precision,
                           pic_particles *p, const double *const *E_dev,
                           double qmdt, double dt, const pic_push_params *params,
                           const int64_t *bin_start_dev, uint32_t *bin_dev, double *Ep_dev,
                           void *stream);

/*
 * Scratch bytes needed by pic_rebin / pic_deposit / pic_step for n particles
 * (the FP32 form of pic_step also keeps the new bins there).  0 for invalid
 * arguments.
 */
size_t pic_scratch_bytes(const pic_tree *tree, int64_t n, int32_t scheme, int32_t precision);

/*
 * The deposit above for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments and result as pic_deposit (the same kernels in
 * the same order, so rho is bit-identical), without the scratch argument:
 * the per-bin partials live in a device-resident array of
 * PIC_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends.  The call allocates nothing (no hipMalloc, no
 * hipFree; kernel timing is off during it).  Limit: the partials take
 * n_bins * 8 * (2^dim for PIT, 3^dim for PIDT) bytes; trees needing more than
 * PIC_NOALLOC_SCRATCH_BYTES get PIC_E_SCRATCH (every 2D tree up to depth 6,
 * 3D PIT trees up to depth 4 and 3D PIDT trees up to depth 3 fit).  The array is looked up for the device that
 * is current at the call; `stream` must belong to it.  Every call on a GPU
 * shares that GPU's array, so calls that overlap on one GPU (other streams,
 * other host threads) race; calls ordered on one stream do not.  Nothing in
 * the array needs to start at zero: each call writes every partial it reads.
 */
#define PIC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
pic_status pic_deposit_noalloc(const pic_tree *tree, int32_t scheme, int32_t precision,
                               const pic_particles *p, const int64_t *bin_start_dev, const double *q_dev,
                               double q_uniform, double *rho_dev, void *stream);

/*
 * Re-bin statistics (paper Sec. 6.1: lifts per particle and time step).  In
 * the paper's PIT a particle that leaves its leaf is lifted towards the root
 * until a cell covers it and dropped from there into its new leaf, so a
 * particle moving from leaf a to leaf b is lifted level(a) - level(c) times,
 * c the coarsest common ancestor of a and b ("n levels = n lifts").  For PIDT
 * the same count is taken in the dual tree (dual cells of a k = 3 tree nest,
 * Sec. 4.1): c is the coarsest dual cell holding the old and the new one.
 * Device record of 64-bit counters, nullable wherever it is accepted.  The
 * calls ADD to it (integer atomics, so the result is deterministic); zero it
 * once and it accumulates over steps.  Layout:
 *   particles   particles counted (n per call);
 *   movers      particles whose new bin differs from their old one;
 *   lifts       sum of the lift counts (0 for particles that stay);
 *   max_tunnel  largest periodic max-norm distance, in finest cells of the
 *               instance, between a particle's old and new bin anchor (leaf
 *               lower corner for PIT, vertex position for PIDT); this is the
 *               maximum only, the other fields are sums;
 *   lift_hist   particles by lift count (entry 0: particles that stayed; the
 *               last entry also counts larger counts).
 */
#define PIC_STATS_LEVELS 20
typedef struct {
    uint64_t particles;
    uint64_t movers;
    uint64_t lifts;
    uint64_t max_tunnel;
    uint64_t lift_hist[PIC_STATS_LEVELS];
} pic_rebin_stats;

/*
 * Re-bin (paper Sec. 5: after the move every particle is held by the grid
 * entity covering it; Theorems 1 and 2; "bucket sort" into children).
 * Output order: bins ascending; inside a bin first the particles that were
 * already in it (in their old order), then the ones that arrived (in their
 * old order).  When old_bin_start_dev is NULL the input is unsorted and every
 * particle counts as arriving.
 *   new_bin_dev        n uint32 bins (from pic_gather_push or pic_locate).
 *   old_bin_start_dev  n_bins+1 int64 offsets of the input order, or NULL.
 *   n_cols, cols_in_dev, cols_out_dev, col_bytes: columns permuted together
 *                      (element size 4 or 8 bytes); outputs must not alias
 *                      inputs.
 *   new_bin_start_dev  receives n_bins+1 int64 offsets of the output.
 *   stats_dev          nullable pic_rebin_stats record the call adds to (needs
 *                      old_bin_start_dev; PIC_E_ARG without it).
 */
pic_status pic_rebin(const pic_tree *tree, int32_t scheme, int64_t n,
                     const uint32_t *new_bin_dev, const int64_t *old_bin_start_dev,
                     int32_t n_cols, void *const *cols_in_dev, void *const *cols_out_dev,
                     const int32_t *col_bytes, int64_t *new_bin_start_dev,
                     void *scratch_dev, size_t scratch_bytes, pic_rebin_stats *stats_dev, void *stream);

/*
 * Deposit (paper Sec. 3 step 1): rho_v = sum_p q_p w_v(x_p) for a sorted set
 * (bin_start_dev from pic_rebin for the same scheme).  rho_dev receives
 * n_vertices doubles (vertex charge, overwritten).  q_dev: per-particle
 * charge (n doubles) or NULL for q_uniform.  No floating-point atomics: each
 * vertex sums its contributions in a fixed order.  FP32 form: per bin, FP32
 * compensated (Kahan) sums, then FP64 over lanes and incident bins.
 */
pic_status pic_deposit(const pic_tree *tree, int32_t scheme, int32_t precision,
                       const pic_particles *p, const int64_t *bin_start_dev,
                       const double *q_dev, double q_uniform, double *rho_dev,
                       void *scratch_dev, size_t scratch_bytes, void *stream);

/*
 * One whole step in a single call: the same result as pic_gather_push, then
 * pic_rebin (in -> out) and pic_deposit (on out) (paper Sec. 3 steps 1, 3, 4;
 * Sec. 5 re-binning).  `in` stays unchanged (unless the tree's knob
 * "key_stores" makes the key pass store the pushed state there, in the old
 * order: by default the FP32 form of 3D trees): a key pass pushes every
 * particle and writes its key 2 * new bin + arrived; a group pass ranks every particle among the particles of its tile with the
 * same key, in tile order; a scan and a placement give every run (tile, key)
 * its destination; an emit pass pushes each particle again (the same
 * arithmetic, so the same state and bin) and writes it to its run's
 * destination plus its rank, in tile-sorted order through LDS.  Then the
 * deposit on `out`.
 *   in                 sorted set with offsets bin_start_dev.
 *   extra_in/out       n_extra further columns (4 or 8 bytes) carried along.
 *   q_column           index of the per-particle charge among the extra
 *                      columns (8-byte), or -1 to use q_uniform.
 *   out                receives the re-binned set; new_bin_start_dev its
 *                      offsets; rho_dev the vertex charge.
 *   stats_dev          nullable pic_rebin_stats record the call adds to.
 * Scratch: pic_scratch_bytes().  E_p is not produced.
 */
pic_status pic_step(const pic_tree *tree, int32_t scheme, int32_t precision, pic_particles *in,
                    const int64_t *bin_start_dev, const double *const *E_dev, double qmdt, double dt,
                    const pic_push_params *params, int32_t n_extra, void *const *extra_in_dev,
                    void *const *extra_out_dev, const int32_t *extra_bytes, int32_t q_column, double q_uniform,
                    pic_particles *out, int64_t *new_bin_start_dev, double *rho_dev, void *scratch_dev,
                    size_t scratch_bytes, pic_rebin_stats *stats_dev, void *stream);

/*
 * Convert a particle set between the FP64 form and the FP32 offset form
 * (trees whose instances are all regular with Peano rank tables).  p must
 * carry both x, v and off, u.  dt: the step the FP32 velocity is scaled by
 * (u = v dt 3^L), or per instance through params->dt_dev.
 *   to_precision PIC_F32_OFFSET: from x, v (any order) writes off = fl32(x 3^L
 *                - I), u = fl32(v dt 3^L) and, in bin_dev, each particle's bin
 *                in the FP32 form (rounding can carry a particle to the next
 *                cell, so re-bin before stepping: pic_rebin with the old
 *                offsets keeps all others in place).
 *   to_precision PIC_F64: from off, u of a sorted set (bin_start_dev) writes
 *                x = (cell + off) / 3^L, v = u / (dt 3^L).
 */
pic_status pic_convert(const pic_tree *tree, int32_t scheme, int32_t to_precision, pic_particles *p, double dt,
                       const pic_push_params *params, const int64_t *bin_start_dev, uint32_t *bin_dev,
                       void *stream);

/* ------------------------------------------------------- measurement aids */

/*
 * Stream benchmark of the paper's evaluation (Sec. 6.2, stream-like particle
 * throughput): every particle moves by one explicit Euler step x <- x + v dt
 * and is reflected at the walls of the unit box (x -> -x below 0, 2 - x
 * above 1, with v negated), with no grid.  x_dev, v_dev: dim pointers to n
 * doubles each, updated in place.  Used to calibrate the achievable HBM
 * bandwidth of structure-of-arrays particle streams.
 */
pic_status pic_stream_push(int32_t dim, int64_t n, double *const *x_dev, double *const *v_dev, double dt,
                           void *stream);

/*
 * Kernel timing.  While enabled, every kernel the library launches is
 * bracketed by two HIP events recorded on its launch stream.
 * pic_profile_read waits for the recorded events, writes up to max_entries
 * per-kernel totals (name, launch count, summed milliseconds) to `out`
 * (may be NULL), forgets them, and returns the number of distinct kernels.
 */
typedef struct {
    char name[48];
    int64_t launches;
    double total_ms;
} pic_kernel_time;

pic_status pic_profile_enable(int32_t on);

/*
 * Restricts timing to launches of one kernel, named as in pic_kernel_time
 * (e.g. "step_move"); NULL or "" times every kernel again.  Lets a caller time
 * one kernel inside a measured region with two events per launch.
 */
pic_status pic_profile_only(const char *name);

/*
 * Launch-shape knobs, for the autotuner.  Every tree carries its own set:
 * pic_tree_tune_set / pic_tree_tune_get change and read the knobs of one
 * tree (and so every call made with it afterwards); pic_tune_set /
 * pic_tune_get change and read the process defaults, which a tree copies
 * when it is created.  Names and values:
 *   "rebin_tile"    particles per rebin tile, 2048 or 4096 (default 2048);
 *   "rebin_radix"   bits per LDS radix pass of the tile sort, 4 or 5 (default 4);
 *   "scatter_mode"  0 = records staged through LDS, 1 = gathered straight from
 *                   the tile (default 0);
 *   "scatter_nt"    1 = non-temporal stores for the re-binned records (default 0);
 *   "scatter_group" columns a scatter thread holds in registers, 1, 2 or 4 (default 4);
 *   "deposit_lanes" lanes that reduce one bin in the FP64 deposit, 16, 32 or 64, or
 *                   0 = 32 for 3D trees and 64 for 2D ones (default 0);
 *   "deposit_bpw"   bins such a lane group takes one after the other, 1 or 2 (default 1);
 *   "deposit_batch" particles a bin's lane group takes per round in the FP64
 *                   deposit, 64 or 256 (default 64; the FP32 deposit takes 256);
 *   "step_tile"     particles per tile of pic_step's ranking and writing passes,
 *                   1024, 2048 or 4096, or 0 = 4096 for 3D trees with at most 256
 *                   particles per bin on average and 2048 otherwise (default 0;
 *                   4096-particle tiles stage one column at a time and ignore
 *                   step_fuse and emit_deposit; the FP32 form takes 4096 where
 *                   the FP64 form would, 2048 otherwise);
 *   "xcd_tiles"     1 = the tiles of pic_step's writing pass are dealt to the chip's
 *                   8 XCDs in contiguous chunks, 0 = in block order (default 1);
 *   "emit_threads"  threads per block of that pass, 512 or 1024 (default 1024);
 *   "step_fuse"     1 = pic_step's FP64 key pass and tile ranking run as one kernel
 *                   (ranking by matching), 0 = as a key pass that writes the keys and
 *                   a ranking pass; 2 = 1 for PIT on 2D single trees whose instances
 *                   are regular, unless key_stores is 1, else 0 (default 2);
 *   "key_stores"    1 = pic_step's key pass stores the pushed state back into `in`
 *                   (x, v or off, u, in the old order) and the writing pass only
 *                   moves it; 0 = the writing pass pushes again and `in` stays
 *                   unchanged; 2 = 1 for the FP32 form of 3D trees, else 0
 *                   (default 2; step_fuse 1 pushes again in any case);
 *   "group_match"   pic_step's ranking pass (step_fuse 0): 0 = every lane tags and
 *                   masks its table slot; 1 = lanes of equal keys found by
 *                   wavefront ballots, one table access per distinct key
 *                   (default 0);
 *   "emit_deposit"  1 = for 2D single trees whose instances are regular and a uniform
 *                   charge, pic_step's writing pass sums each run's weights while
 *                   the run is in LDS and the deposit only adds runs per bin; 0 = the
 *                   deposit reads the re-binned positions again; 2 = 1 for PIT and
 *                   0 for PIDT, whose nine-weight stencil costs the writing pass
 *                   more than the second read (default 2);
 *   "regular_tables" (process default only) 1 = trees created afterwards get Peano
 *                   rank tables for their regular instances (up to 2^21 cells per
 *                   level), which the arithmetic kernels and the FP32 form use;
 *                   0 = none, every tree takes the descent kernels (default 1).
 * Every setting gives the same bins, order and particle state; "deposit_lanes"
 * and "emit_deposit" change the order of the deposit's sums, so the charge
 * differs in rounding only (far inside the stated tolerance).  pic_scratch_bytes covers all settings.
 * Affects calls enqueued afterwards.  Unknown names or values: PIC_E_ARG
 * (pic_tune_get returns -1).
 */
pic_status pic_tune_set(const char *name, int64_t value);
int64_t pic_tune_get(const char *name);
pic_status pic_tree_tune_set(pic_tree *tree, const char *name, int64_t value);
int64_t pic_tree_tune_get(const pic_tree *tree, const char *name);
int32_t pic_profile_read(pic_kernel_time *out, int32_t max_entries);

/* ------------------------------------------- particle-handling benchmark
 *
 * The workload of the paper's results section (Sec. 6 setup): the field
 * solve and the particle-grid coupling are left out, every particle streams
 * freely, the walls reflect, a fixed number of artificial flops can be
 * imposed on every move, and the tree follows the particles: a leaf holding
 * more than ppc particles is refined, children that together hold at most
 * ppc are removed.  A step is pic_free_stream, then pic_rebin (whose
 * statistics give the lifts per particle, Sec. 6.1); an adaptation is
 * pic_leaf_counts (or the bin offsets of a PIT-sorted set), pic_tree_adapt,
 * pic_tree_create on the returned masks, then pic_locate and pic_rebin of
 * the particles against the new tree (the paper's remark in Sec. 5 that
 * added and removed nodes re-sort particles by the same mechanism).
 */

/*
 * Free streaming, in place: per axis x <- x + v dt, then the wall rule:
 *   PIC_PERIODIC    x <- x - floor(x), 1.0 -> 0.0;
 *   PIC_REFLECTING  below 0: x <- -x; at or above 1: x <- 2 - x; either way
 *                   v <- -v for that axis; a landing exactly on 1 is put at
 *                   the largest double below 1.
 * A move that one mirror cannot bring back into [0,1) (|v dt| >= 1 towards
 * a wall) or a non-finite value sets PIC_E_RANGE / PIC_E_NONFINITE in the
 * status word (the particle is clamped into the box).  `flops` artificial
 * floating-point operations (a dependent multiply-add chain whose result is
 * discarded; even values, 0 to 2^20) are carried out per particle.  The new
 * bin of every particle under `scheme` is written to bin_dev (n uint32).
 * dt for a single tree; per instance from params->dt_dev when set (params
 * may be NULL; its qmdt_dev is ignored).  FP64 form only (PIC_E_ARG
 * otherwise).  x and v change bit-identically to a serial IEEE evaluation
 * of the same formulas.
 */
pic_status pic_free_stream(const pic_tree *tree, int32_t scheme, int32_t precision, pic_particles *p,
                           double dt, const pic_push_params *params, int32_t boundary, int32_t flops,
                           uint32_t *bin_dev, void *stream);

/*
 * The same step as pic_free_stream then pic_rebin (in -> out), in the
 * passes of pic_step: a key pass streams every particle (with the
 * artificial flops) and writes its key 2 * new bin + arrived, the ranking,
 * scan and placement give every (tile, key) run its destination, and a
 * writing pass streams each particle again (the same arithmetic without the
 * flops, so the same state and bin) and writes it there; no deposit.  The
 * result (out, new_bin_start, stats) equals the two calls' bit for bit.
 * Single trees (PIC_E_ARG for forests), FP64 form; the arguments as in
 * pic_free_stream and pic_step (`in` stays unchanged unless the tree's knob
 * "key_stores" is 1).  Scratch: pic_scratch_bytes().
 */
pic_status pic_stream_step(const pic_tree *tree, int32_t scheme, pic_particles *in, const int64_t *bin_start_dev,
                           double dt, int32_t boundary, int32_t flops, int32_t n_extra, void *const *extra_in_dev,
                           void *const *extra_out_dev, const int32_t *extra_bytes, pic_particles *out,
                           int64_t *new_bin_start_dev, void *scratch_dev, size_t scratch_bytes,
                           pic_rebin_stats *stats_dev, void *stream);

/*
 * Particles per leaf: count_dev (device, forest-wide leaf count entries of
 * uint64) is overwritten with the number of particles of p whose position
 * lies in each leaf (the PIT bin, Theorem 1).  Any order of p.  For a set
 * sorted into PIT bins the bin offsets give the same numbers.
 */
pic_status pic_leaf_counts(const pic_tree *tree, const pic_particles *p, uint64_t *count_dev, void *stream);

/*
 * One ppc-driven adaptation of a single tree (host only, synchronous):
 *   - a leaf whose count exceeds ppc is refined if its level is below
 *     max_level;
 *   - a refined cell other than the root whose 3^d children are all leaves
 *     (none of them refined by the rule above) holding together at most ppc
 *     particles loses its children.
 * leaf_count: host, one int64 per leaf in leaf-rank order.  The result is
 * written as the refine masks pic_tree_create takes (levels 0 .. new
 * max_level-1, (3^l)^d bytes each, 1 = refined; 0 for every cell that does
 * not exist): *new_max_level and *masks_len (bytes) are always set; masks
 * may be NULL with masks_cap 0 to ask for the size, and PIC_E_CAPACITY is
 * returned when masks_cap is below *masks_len.  One rule application per
 * call (an overfull leaf gains one level per call).  PIC_E_ARG for forests,
 * negative ppc or a max_level outside the tree limits; PIC_E_CAPACITY when
 * the dense state of the deepest level the result can reach ((3^l)^d bytes)
 * would exceed 16 GiB; PIC_E_MEMORY when the host heap is exhausted.
 */
pic_status pic_tree_adapt(const pic_tree *tree, const int64_t *leaf_count, int64_t ppc, int32_t max_level,
                          uint8_t *masks, size_t masks_cap, size_t *masks_len, int32_t *new_max_level);

/*
 * raPIDT's analysed tree attribute (paper Sec. 5.4, Eq. (vmax)) of a single
 * tree for a set sorted into `scheme` bins (bin_start_dev):
 *   leaf c:    v_max(c) = the largest |v_k| over the particles of c (PIT) or
 *              of the dual cells of c's 2^d corners at c's level (PIDT);
 *   refined c: v_max(c) = the largest v_max of its children.
 * vmax_dev (device) receives one double per cell position of levels 0..L in
 * the layout of the refine masks, level after level ((3^l)^d positions,
 * lexicographic): (3^(d(L+1)) - 1) / (3^d - 1) entries, 0 where no cell
 * exists.  quiet_dev (device, nullable, same count of uint8) receives the
 * paper's predicate v_max(c) * dt <= h(c) = 1/3^l per existing cell (1:
 * no particle of c can move by a cell width of c in one step), 0 where no
 * cell exists.  The maxima are exact and do not depend on launch order.
 * scratch: n_bins doubles (pic_scratch_bytes covers it).  PIC_E_ARG for
 * forests.
 */
pic_status pic_vmax(const pic_tree *tree, int32_t scheme, const pic_particles *p, const int64_t *bin_start_dev,
                    double dt, double *vmax_dev, uint8_t *quiet_dev, void *scratch, size_t scratch_bytes,
                    void *stream);

#ifdef __cplusplus
}
#endif

#endif /* PIC_H */
