// Device-side descriptors and kernel launchers of librqc (gfx950).
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>

#include "host.hpp"

namespace rqc {

// Values of the projected variables of one slice group (fixed output bits and
// looped sliced legs), one bit each.
struct ProjVals {
    uint64_t w[4];
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
    int m_fast = 0; // tile order: m fastest (set by the launcher)
    int ksplit = 1; // > 1: K in ksplit ranges, partial sums in W ([range][batch][m][n]), then added in order
    float2 *W = nullptr;
    int c_ins_pos = 0, c_ins_bits = 0; // C layout: the low c_ins_bits M bits sit at N bit c_ins_pos
};

void launch_leaf_select(const float2 *full, float2 *leafbuf, const LeafSel *d_sel, int n_leaves,
                        ProjVals vals, hipStream_t s);
// d_trees: the first of n_trees subtrees to run; cache: the slice group's
// global-cache block (subtree roots kept there), or null
void launch_small_trees(const SmallStep *d_steps, const SmallTree *d_trees, int n_trees, int lds_elems,
                        const float2 *leafbuf, float2 *arena, float2 *cache, hipStream_t s);
// d_maps: the op's SM_COUNT bit maps in device memory; w: the op's scratch
// (long form only, else null); b2: the second B of a fused pair (else null)
void launch_stream(const StreamOp &op, const BitMap *d_maps, const float2 *a, const float2 *b, float2 *c,
                   float2 *w, const float2 *b2, hipStream_t s);
// d_desc: the permute descriptor in device memory
void launch_permute(const PermDesc *d_desc, int64_t n_tiles, const float2 *src, float2 *dst, hipStream_t s);
// the same with the descriptor in the kernel arguments
void launch_permute_value(const PermDesc &d, const float2 *src, float2 *dst, hipStream_t s);
// precision: rqc_precision; amax: two device words of scratch (fp16 scaling)
void launch_gemm(const GemmArgs &g, int precision, unsigned *amax, hipStream_t s);
// d_maps[0]: open index -> root offset, d_maps[1]: batched slice index -> root offset
void launch_accumulate(const float2 *root, const BitMap *d_maps, int n_open, int n_batched, double2 *acc,
                       hipStream_t s);
void launch_zero(double2 *acc, int64_t n, hipStream_t s);
void launch_finalize(const double2 *acc, int64_t n, double scale, float2 *out, double2 *out64,
                     hipStream_t s);

// sampler: `work` is device memory of at least sampler_scratch_bytes(items,
// batches, n_open) bytes, where items = pick_steps in pick mode, else
// n_batches * 2^(n_open - log2_na); fixed and open_q are host arrays.  The
// call synchronises s before returning.
size_t sampler_scratch_bytes(int64_t n_items, int64_t n_batches, int n_open);
hipError_t run_sampler(const float2 *amps, const uint64_t *fixed, int64_t n_batches, const int32_t *open_q,
                       int n_open, int log2_na, int n_qubits, double alpha, double f_norm, uint64_t seed,
                       uint64_t base, int64_t pick_steps, int64_t n_samples, uint64_t *out,
                       int64_t *n_out, rqc_sample_stats *stats, void *work, hipStream_t s);

// Top-count selection (select.hip): `work` is device memory of at least
// select_scratch_bytes(2^n_open) bytes; open_q is a host array.  Asynchronous.
size_t select_scratch_bytes(int64_t n);
// FP64 probability sums of n_rows rows of row_len amplitudes, and their XEB
// (Eq. (1)) when xeb is not null; `work` is device memory of at least
// prob_sums_scratch_bytes(n_rows, row_len) bytes.  n_rows * ceil(row_len /
// 8192) < 2^31.  Asynchronous.
size_t prob_sums_scratch_bytes(int64_t n_rows, int64_t row_len);
void launch_prob_sums(const float2 *amps, int64_t n_rows, int64_t row_len, int n_qubits, double *sums, double *xeb,
                      void *work, hipStream_t s);
void launch_select_top(const float2 *amps, int n_open, const int32_t *open_q, uint64_t fixed, int64_t count,
                       uint64_t *out, void *work, hipStream_t s);

// The fixed device array of rqc_rejection_sample_static on the current device
// (its address from hipGetSymbolAddress, looked up once per device) and the
// lock that serialises the calls using it on that device.
constexpr int kMaxDevices = 64;
hipError_t static_scratch(void **ptr, std::mutex **call_mu);

} // namespace rqc
