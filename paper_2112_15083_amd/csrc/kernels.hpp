// Device-side descriptors and kernel launchers of librqc (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include "host.hpp"

namespace rqc {

// Values of the projected variables of one slice group (fixed output bits and
// looped sliced legs), one bit each.
struct ProjVals {
    uint64_t w[4];
};

// Leaf selection: copy a leaf's sub-tensor with its projected legs fixed.
struct LeafSel {
    int64_t src;        // offset of the full leaf in the leaf store (complex64 elements)
    int64_t dst;        // offset of the projected leaf in the leaf buffer
    int32_t n_free;     // legs kept
    int32_t n_proj;     // legs fixed by projected values
    uint8_t free_pos[4];  // full-layout bit of kept leg j
    uint8_t proj_pos[4];  // full-layout bit of projected leg j
    int16_t proj_idx[4];  // projected-variable index of projected leg j
};

// Tiled bit permutation: dst[P(x)] = src[x].
struct PermDesc {
    BitMap tile_src, tile_dst; // tile index -> source / destination base offset
    BitMap rd;                 // read-order index -> source offset inside the tile
    BitMap wr_lds, wr_dst;     // write-order index -> LDS slot / destination offset
    int32_t tile_log;          // log2 elements per tile
    int64_t n_tiles;
};
PermDesc make_perm_desc(int r, const std::vector<int> &perm);

struct GemmArgs {
    const float2 *A;
    const float2 *B;
    float2 *C;
    int64_t batch, M, N, K;
    int64_t sa, sb, sc;
    int a_kfast, b_nfast;
};

void launch_leaf_select(const float2 *full, float2 *leafbuf, const LeafSel *d_sel, int n_leaves,
                        ProjVals vals, hipStream_t s);
void launch_small_trees(const SmallStep *d_steps, const SmallTree *d_trees, int n_trees, int lds_elems,
                        const float2 *leafbuf, float2 *arena, hipStream_t s);
void launch_stream(const StreamOp &op, const float2 *a, const float2 *b, float2 *c, hipStream_t s);
void launch_permute(const PermDesc &d, const float2 *src, float2 *dst, hipStream_t s);
void launch_gemm(const GemmArgs &g, int precision, hipStream_t s);
void launch_accumulate(const float2 *root, const BitMap &open_map, const BitMap &slice_map, int n_open,
                       int n_batched, double2 *acc, hipStream_t s);
void launch_zero(double2 *acc, int64_t n, hipStream_t s);
void launch_finalize(const double2 *acc, int64_t n, double scale, float2 *out, double2 *out64,
                     hipStream_t s);

// sampler
struct SampleOut {
    uint64_t bits;
};
hipError_t run_sampler(const float2 *amps, const uint64_t *d_fixed, int64_t n_batches, const int32_t *d_open,
                       int n_open, int log2_na, int n_qubits, double alpha, double f_norm, uint64_t seed,
                       uint64_t base, int64_t pick_steps, int64_t n_samples, uint64_t *out,
                       int64_t *n_out, rqc_sample_stats *stats, hipStream_t s);

} // namespace rqc
