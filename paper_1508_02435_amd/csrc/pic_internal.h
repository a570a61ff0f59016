// pic_internal.h -- device-side layout of the linearised spacetree and the
// integer helpers shared by the host builder and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define PIC_MAX_LEVEL 18      // 3^18 < 2^29: finest coordinates fit 29 bits
#define PIC_LDS_NODES 4096    // descent-table entries staged in LDS (16 KiB)
#define PIC_STATS_LEVELS 20   // lift-count histogram entries of the re-bin statistics

// status bits in the device status word (sticky, OR-ed by kernels)
#define PIC_DEV_NONFINITE 1u
#define PIC_DEV_RANGE 2u

namespace pic {

// ---------------------------------------------------------------------------
// Exact floor(n / 3^e) for n < 2^30 by multiply-high (Granlund-Montgomery):
// with k = 30 + ceil(log2 3^e) and M = ceil(2^k / 3^e),
// floor(n * M / 2^k) = floor(n / 3^e) for every n < 2^30, and n*M < 2^62.
// ---------------------------------------------------------------------------
struct DivMagic {
    uint64_t mul;
    uint32_t shift;
};

constexpr uint64_t pow3_u64(int e) { return e == 0 ? 1ull : 3ull * pow3_u64(e - 1); }
constexpr int ceil_log2_u64(uint64_t v) {
    int r = 0;
    while ((1ull << r) < v) ++r;
    return r;
}
constexpr DivMagic make_magic(int e) {
    return DivMagic{((1ull << (30 + ceil_log2_u64(pow3_u64(e)))) + pow3_u64(e) - 1) / pow3_u64(e),
                    (uint32_t)(30 + ceil_log2_u64(pow3_u64(e)))};
}

__host__ __device__ inline uint32_t pow3_u32(int e) {
    uint32_t r = 1;
    for (int i = 0; i < e; ++i) r *= 3u;
    return r;
}

// Peano rank of lattice cell a[] over its lowest `nd` base-3 digits.  The
// curve index takes digits from the most significant down, axes interleaved
// 0..D-1; the digit of axis k is complemented (2-digit) when the digits
// already emitted for the other axes have an odd sum.  Because 3 is odd, the
// digit sum of a base-3 number has the parity of the number itself, so the
// parity of "all digits of axis j at or above position t" is just
// (a_j / 3^t) & 1.  The loop therefore runs from the least significant digit
// up and needs no prefix bookkeeping; digits above `nd` only enter through
// those parities, which makes the result the rank inside the uniform subtree
// whose root sits nd levels above the cell.
template <int D>
__host__ __device__ inline uint32_t peano_low(const uint32_t *a, int nd) {
    uint32_t q[D];
#pragma unroll
    for (int k = 0; k < D; ++k) q[k] = a[k];
    uint32_t key = 0, mult = 1;
    for (int t = 0; t < nd; ++t) {
        uint32_t qn[D], dig[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            qn[k] = q[k] / 3u;
            dig[k] = q[k] - 3u * qn[k];
        }
#pragma unroll
        for (int k = D - 1; k >= 0; --k) {
            uint32_t par = 0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                if (j < k) par ^= q[j] & 1u;       // axis j already emitted this digit
                else if (j > k) par ^= qn[j] & 1u; // axis j emits it after k
            }
            uint32_t e = par ? 2u - dig[k] : dig[k];
            key += e * mult;
            mult *= 3u;
        }
#pragma unroll
        for (int k = 0; k < D; ++k) q[k] = qn[k];
    }
    return key;
}

// ---------------------------------------------------------------------------
// One spacetree of a forest, as the kernels see it.
// ---------------------------------------------------------------------------
struct DevInst {
    int32_t L;          // deepest level
    int32_t regular;    // uniformly refined to L: every bin is computed arithmetically
    int32_t S;          // 3^L, finest cells per axis
    int32_t node_root;  // forest-wide index of this instance's root in node_child
    int32_t leaf_off, n_leaves;
    int32_t vtx_off, n_vtx;
    int32_t pidt_off, n_pidt;
    int32_t lds_nodes;  // leading descent entries of this instance held in LDS (single tree)
    int32_t ptab;       // regular instances: offset of the Peano rank table of their level, else -1
    double Sd;          // (double)S
    double rinv[PIC_MAX_LEVEL + 1];  // fl(1 / 3^(L-l)) indexed by leaf level l
};

// Device tables of the whole forest (pointers into the caller's tree buffer).
struct DevTree {
    int32_t dim, n_inst;
    int32_t all_regular, pad0;
    int64_t n_leaves, n_vtx, n_pidt, n_nodes;
    const DevInst *inst;        // n_inst
    const int32_t *node_child;  // >= 0: first child (3^d lexicographic slots); < 0: -(u+1) uniform subtree u
    const uint32_t *uni_base;   // forest-wide leaf rank of the uniform subtree's first leaf
    const uint32_t *uni_meta;   // root level | depth << 8
    const uint8_t *leaf_level;  // n_leaves
    const int32_t *leaf_vtx;    // n_leaves * 2^d forest-wide vertex ids
    const int32_t *leaf_pidt;   // n_leaves * 2^d forest-wide PIDT bins
    const uint8_t *pidt_level;  // n_pidt
    const int32_t *leaf_inst;   // n_leaves: instance of each leaf
    const int32_t *pidt_inst;   // n_pidt
    const int32_t *vtx_inst;    // n_vtx
    const int32_t *vinc_ptr;    // n_vtx + 1: CSR vertex -> (leaf * 2^d + corner), ascending
    const int32_t *vinc;
    const int32_t *vpinc_ptr;   // n_vtx + 1: CSR vertex -> (pidt bin * 3^d + stencil slot), ascending
    const int32_t *vpinc;
    const uint32_t *peano_tab;  // per level of regular instances: Peano rank of finest cell c0 + S c1 (+ S^2 c2)
    const uint32_t *cell_tab;   // the inverse: lattice index c0 + S c1 (+ S^2 c2) of each Peano rank
    const uint32_t *leaf_coord; // n_leaves * dim: leaf coordinates at the leaf's own level
    const uint32_t *pidt_b;     // n_pidt * dim: vertex coordinates at the bin's level
    uint32_t *status;           // sticky device status word
};

}  // namespace pic
