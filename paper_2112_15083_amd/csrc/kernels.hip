// HIP kernels of librqc for gfx950 (CDNA4, wave64).
//
//   k_leaf_select   slice / fixed-bit selection of the leaf tensors (Sec. I.C,
//                   step 1: the sliced vertices take one value per slice)
//   k_small_trees   one workgroup per small subtree, intermediates in LDS
//   k_stream        streaming contraction with a short contracted dimension
//   k_permute       LDS-tiled bit permutation of a tensor (coalesced both ways)
//   k_cgemm_f32     complex GEMM on FP32 MFMA (v_mfma_f32_32x32x2f32)
//   k_accumulate    FP64 cross-slice sum in a fixed slice order (Sec. I.C)
//   k_finalize      1/sqrt(F) normalisation and complex64 output (Sec. I.C, step 2)
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "kernels.hpp"

namespace rqc {

__device__ __forceinline__ int64_t map_apply(const BitMap &m, int64_t x) {
    int64_t r = 0;
    for (int i = 0; i < m.n; i++) {
        const uint32_t w = m.run[i];
        r |= ((x >> (w & 255u)) & ((1LL << ((w >> 8) & 255u)) - 1)) << (w >> 16);
    }
    return r;
}

__device__ __forceinline__ void cmac(float2 &acc, float2 a, float2 b) {
    acc.x += a.x * b.x - a.y * b.y;
    acc.y += a.x * b.y + a.y * b.x;
}

// ------------------------------------------------------------------ leaf select
__global__ void __launch_bounds__(256) k_leaf_select(const float2 *__restrict__ full, float2 *__restrict__ leafbuf,
                                                     const LeafSel *__restrict__ sel, int n_leaves, ProjVals vals) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int leaf = gid >> 4, e = gid & 15;
    if (leaf >= n_leaves) return;
    const LeafSel &d = sel[leaf];
    if (e >= (1 << d.n_free)) return;
    int64_t src = d.src;
    for (int j = 0; j < d.n_free; j++)
        if ((e >> j) & 1) src += (int64_t)1 << d.free_pos[j];
    for (int j = 0; j < d.n_proj; j++) {
        const int p = d.proj_idx[j];
        if ((vals.w[p >> 6] >> (p & 63)) & 1) src += (int64_t)1 << d.proj_pos[j];
    }
    leafbuf[d.dst + e] = full[src];
}

void launch_leaf_select(const float2 *full, float2 *leafbuf, const LeafSel *d_sel, int n_leaves, ProjVals vals,
                        hipStream_t s) {
    if (n_leaves <= 0) return;
    const int threads = 256;
    const int blocks = (n_leaves * 16 + threads - 1) / threads;
    hipLaunchKernelGGL(k_leaf_select, dim3(blocks), dim3(threads), 0, s, full, leafbuf, d_sel, n_leaves, vals);
}

// ------------------------------------------------------------------ small subtrees
__global__ void __launch_bounds__(256) k_small_trees(const SmallStep *__restrict__ steps,
                                                     const SmallTree *__restrict__ trees,
                                                     const float2 *__restrict__ leafbuf, float2 *__restrict__ arena,
                                                     float2 *__restrict__ cache) {
    extern __shared__ float2 lds[];
    const SmallTree t = trees[blockIdx.x];
    for (int s = t.first_step; s < t.first_step + t.n_steps; s++) {
        const SmallStep &st = steps[s];
        const float2 *A = st.a_kind == 0 ? lds + st.a_off : (st.a_kind == 1 ? leafbuf + st.a_off : arena + st.a_off);
        const float2 *B = st.b_kind == 0 ? lds + st.b_off : (st.b_kind == 1 ? leafbuf + st.b_off : arena + st.b_off);
        float2 *C = st.c_kind == 0 ? lds + st.c_off : (st.c_kind == 3 ? cache : arena) + st.c_off;
        const int nC = 1 << st.rc, nK = 1 << st.kc;
        for (int x = threadIdx.x; x < nC; x += blockDim.x) {
            const int64_t ax = map_apply(st.ax, x), bx = map_apply(st.bx, x);
            float2 acc = make_float2(0.f, 0.f);
            for (int y = 0; y < nK; y++) cmac(acc, A[ax + map_apply(st.ay, y)], B[bx + map_apply(st.by, y)]);
            C[x] = acc;
        }
        __syncthreads();
    }
}

void launch_small_trees(const SmallStep *d_steps, const SmallTree *d_trees, int n_trees, int lds_elems,
                        const float2 *leafbuf, float2 *arena, float2 *cache, hipStream_t s) {
    if (n_trees <= 0) return;
    hipLaunchKernelGGL(k_small_trees, dim3(n_trees), dim3(256), (size_t)lds_elems * sizeof(float2), s, d_steps,
                       d_trees, leafbuf, arena, cache);
}

// ------------------------------------------------------------------ streaming contraction
// General form for long contracted or new-leg dimensions: one output per
// thread and iteration, contracted offsets tabulated in LDS (low 10 bits) and
// mapped per high part.
__global__ void __launch_bounds__(256) k_stream_gen(const float2 *__restrict__ A, const float2 *__restrict__ B,
                                                    float2 *__restrict__ C, const BitMap *__restrict__ maps, int nr,
                                                    int kc, int nf) {
    __shared__ int64_t tyA[1024], tyB[1024];
    const int tid = threadIdx.x;
    const int ylo = kc < 10 ? kc : 10;
    const int nylo = 1 << ylo;
    const int64_t nyhi = (int64_t)1 << (kc - ylo);
    for (int i = tid; i < nylo; i += blockDim.x) {
        tyA[i] = map_apply(maps[SM_YA], i);
        tyB[i] = map_apply(maps[SM_YB], i);
    }
    __syncthreads();
    const int64_t n = (int64_t)1 << (nr + nf);
    const int64_t nfm = ((int64_t)1 << nf) - 1;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + tid; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t f = x & nfm, r = x >> nf;
        const int64_t ab = map_apply(maps[SM_RA], r);
        const int64_t bb = map_apply(maps[SM_RB], r) + map_apply(maps[SM_FB], f);
        float2 acc = make_float2(0.f, 0.f);
        for (int64_t yh = 0; yh < nyhi; yh++) {
            const int64_t ah = ab + map_apply(maps[SM_YA], yh << ylo), bh = bb + map_apply(maps[SM_YB], yh << ylo);
            for (int yl = 0; yl < nylo; yl++) cmac(acc, A[ah + tyA[yl]], B[bh + tyB[yl]]);
        }
        C[map_apply(maps[SM_RC], r) + map_apply(maps[SM_FC], f)] = acc;
    }
}

// LDS-tiled form (see StreamOp): loads and stores follow the memory order of A
// and C, so both are coalesced whatever the leg order; the compute phase reads
// LDS through an XOR swizzle that keeps strided slot patterns conflict-free.
__device__ __forceinline__ int swz(int e) { return e ^ ((e >> 5) & 31); }

template <int KMAX, int FMAX>
__global__ void __launch_bounds__(256) k_stream_tile(const float2 *__restrict__ A, const float2 *__restrict__ B,
                                                     float2 *__restrict__ C, const BitMap *__restrict__ maps, int nr,
                                                     int kc, int nf, int L) {
    constexpr int FA = FMAX > 0 ? FMAX : 1;
    __shared__ float2 TA[2048], TC[2048];
    __shared__ int tyE[KMAX], tfE[FA];
    __shared__ int64_t tyB[KMAX], tfB[FA];
    const int tid = threadIdx.x;
    const int nK = 1 << kc, nF = 1 << nf;
    if (tid < nK) {
        tyE[tid] = (int)map_apply(maps[SM_YE], tid);
        tyB[tid] = map_apply(maps[SM_YB], tid);
    }
    if (FMAX > 0 && tid < nF) {
        tfE[tid] = (int)map_apply(maps[SM_FE], tid);
        tfB[tid] = map_apply(maps[SM_FB], tid);
    }
    const int nA = 1 << (L + kc), nC = 1 << (L + nf), nR = 1 << L;
    int64_t offA[8], offC[8];
#pragma unroll
    for (int k = 0; k < 8; k++) {
        const int e = tid + 256 * k;
        offA[k] = e < nA ? map_apply(maps[SM_EA], e) : 0;
        offC[k] = e < nC ? map_apply(maps[SM_EC], e) : 0;
    }
    const int eR = tid < nR ? (int)map_apply(maps[SM_RE], tid) : 0;
    const int eR2 = tid < nR ? (int)map_apply(maps[SM_RE2], tid) : 0;
    const int64_t bR = tid < nR ? map_apply(maps[SM_RB], tid) : 0;
    __syncthreads();
    const int64_t n_tiles = (int64_t)1 << (nr - L);
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const int64_t r0 = t << L;
        const int64_t ab = map_apply(maps[SM_RA], r0), bb = map_apply(maps[SM_RB], r0) + bR,
                      cb = map_apply(maps[SM_RC], r0);
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int e = tid + 256 * k;
            if (e < nA) TA[swz(e)] = A[ab + offA[k]];
        }
        __syncthreads();
        if (FMAX > 0) {
            // register blocking: one r per thread, all its outputs
            if (tid < nR) {
                float2 a[KMAX];
#pragma unroll
                for (int y = 0; y < KMAX; y++)
                    if (y < nK) a[y] = TA[swz(eR + tyE[y])];
#pragma unroll
                for (int f = 0; f < (FMAX > 0 ? FMAX : 1); f++) {
                    if (f < nF) {
                        float2 acc = make_float2(0.f, 0.f);
                        const float2 *bp = B + bb + tfB[f];
#pragma unroll
                        for (int y = 0; y < KMAX; y++)
                            if (y < nK) cmac(acc, a[y], bp[tyB[y]]);
                        TC[swz(eR2 + tfE[f])] = acc;
                    }
                }
            }
        } else {
            // many new legs: one (r, f) output per thread and iteration
            const int64_t bt = bb - bR;
            for (int o = tid; o < nC; o += 256) {
                const int rl = o & (nR - 1), f = o >> L;
                const int er = (int)map_apply(maps[SM_RE], rl), er2 = (int)map_apply(maps[SM_RE2], rl);
                const float2 *bp = B + bt + map_apply(maps[SM_RB], rl) + map_apply(maps[SM_FB], f);
                float2 acc = make_float2(0.f, 0.f);
                for (int y = 0; y < nK; y++) cmac(acc, TA[swz(er + tyE[y])], bp[tyB[y]]);
                TC[swz(er2 + (int)map_apply(maps[SM_FE], f))] = acc;
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 8; k++) {
            const int e = tid + 256 * k;
            if (e < nC) C[cb + offC[k]] = TC[swz(e)];
        }
    }
}

// Long contracted dimension (2^kc >= 64) with few new legs: one wave per r,
// lanes along the contracted index (y = 64 j + lane), all 2^nf outputs of that
// r accumulated per lane, then summed across the wave by a fixed xor-shuffle
// tree, so the result does not depend on scheduling.
template <int FMAX>
__global__ void __launch_bounds__(256) k_stream_ky(const float2 *__restrict__ A, const float2 *__restrict__ B,
                                                   float2 *__restrict__ C, const BitMap *__restrict__ maps, int nr,
                                                   int kc, int nf) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t r = (int64_t)blockIdx.x * 4 + wave;
    if (r >= ((int64_t)1 << nr)) return;
    const int nF = 1 << nf;
    const int64_t nK = (int64_t)1 << kc;
    const int64_t ab = map_apply(maps[SM_RA], r) + map_apply(maps[SM_YA], lane);
    const int64_t bb = map_apply(maps[SM_RB], r) + map_apply(maps[SM_YB], lane);
    int64_t fb[FMAX];
#pragma unroll
    for (int f = 0; f < FMAX; f++) fb[f] = f < nF ? map_apply(maps[SM_FB], f) : 0;
    float2 acc[FMAX];
#pragma unroll
    for (int f = 0; f < FMAX; f++) acc[f] = make_float2(0.f, 0.f);
    for (int64_t yb = 0; yb < nK; yb += 64) {
        const int64_t ya = map_apply(maps[SM_YA], yb), yb_ = map_apply(maps[SM_YB], yb);
        const float2 a = A[ab + ya];
#pragma unroll
        for (int f = 0; f < FMAX; f++)
            if (f < nF) cmac(acc[f], a, B[bb + yb_ + fb[f]]);
    }
#pragma unroll
    for (int f = 0; f < FMAX; f++) {
        if (f < nF) {
            float2 v = acc[f];
            for (int off = 32; off > 0; off >>= 1) {
                v.x += __shfl_xor(v.x, off, 64);
                v.y += __shfl_xor(v.y, off, 64);
            }
            if (lane == 0) C[map_apply(maps[SM_RC], r) + map_apply(maps[SM_FC], f)] = v;
        }
    }
}

// Short contraction on matrix cores.  Per tile of R = 2^L rows (64..256):
// C[r][f] = sum_y A[r][y] B_r[y][f] with K = 2^KC <= 32 and F = 2^nf <= 64.
// As a real product, [A_re | A_im] interleaved per y (row length 2K) times the
// 2K x 2F block matrix with entries B'[2y+c][2f+d] = (B_re, B_im; -B_im, B_re)
// [c][d] gives C interleaved per f, i.e. the complex rows of C.  Each wave owns
// a quarter of the tile's rows in 16-row blocks and runs them through
// v_mfma_f32_16x16x4f32 with B' held in registers (NC blocks of 16 columns);
// the tile's batch legs are its top two row bits, so a wave's rows share one
// B matrix.  A and C go through LDS row-major ([row][y] with row stride K+1,
// [row][f] with stride F+1) between coalesced HBM reads and writes; the next
// tile's A is loaded into registers while the current one is computed.
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Buffer resource for 16-byte accesses at 32-bit byte offsets from a tile base
// (raw buffer, no stride, full range).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const float2 *base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float2 *>(base), (short)0, -1, 0x00020000);
}

// Waves per SIMD that each instance's register budget is held to (B' takes
// max(1, 2^(KC-1)) * NC registers per lane, the accumulators 4 * NC): four
// wherever B', the accumulators and both A prefetch sets fit 128 registers
// without spilling, else what the instance reaches unconstrained.
constexpr int mx_waves(int KC, int NC) {
    return NC == 8 ? (KC <= 1 ? 3 : KC <= 4 ? 2 : 1)
           : KC == 5 ? (NC <= 2 ? 3 : 2)
           : (KC >= 3 && NC == 4) ? 3 : 4;
}

// WIDE: tiles whose elements span 2^29 or more (tensors of 2^30 elements, 8
// GiB): offsets are held in elements and each access is a global load or
// store at a 64-bit address, instead of a buffer access at a 32-bit byte offset.
template <int KC, int NC, bool WIDE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(mx_waves(KC, NC)))) k_stream_mx(const float2 *__restrict__ A, const float2 *__restrict__ B,
                                                   float2 *__restrict__ C, const BitMap *__restrict__ maps, int nr,
                                                   int nf, int L) {
    // A rows hold (re, im) per y as floats at a stride of RSA = 4 * odd floats,
    // so a wave's operand reads (16 rows by 4 consecutive floats) hit 64
    // distinct banks; C rows hold F complex at a stride of F + 2, so the 4 rows
    // a wave writes per accumulator register start 16 banks apart.
    constexpr int K = 1 << KC, RSA = (K >= 4 ? 2 * K : 8) + 4, KP = RSA / 2;
    constexpr int NT = K >= 2 ? K / 2 : 1; // 4-deep real k steps: 2K / 4
    extern __shared__ float2 lds[];
    const int R = 1 << L, F = 1 << nf, FP = F + 2;
    float2 *TA = lds;
    const float *TAf = reinterpret_cast<const float *>(lds);
    float2 *TC = lds + R * KP;
    float *TCf = reinterpret_cast<float *>(TC);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // Every thread moves 4 pairs of adjacent elements each way as 16-byte
    // accesses (tile bit 0 is tensor bit 0) at 32-bit byte offsets from the
    // tile base; the pair's two LDS slots are packed in one word.  Beyond a
    // tile's size the pair index wraps, so the extra copies read and write
    // identical values: all tile loads and stores are unconditional, which
    // lets the compiler wait for exactly the loads it needs.
    constexpr int CPT = NC == 8 ? 8 : 4; // C pairs per thread (tiles of 2^12 C elements for 2^nf = 64)
    const int hA = (R << KC) >> 1, hC = (R << nf) >> 1;
    uint32_t oA[4], sA[4], oC[CPT], sC[CPT];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int ea = 2 * ((tid + 256 * k) & (hA - 1));
        oA[k] = (uint32_t)map_apply(maps[SM_EA], ea) * (WIDE ? 1u : 8u);
        sA[k] = (uint32_t)(map_apply(maps[SM_ER], ea) * KP + map_apply(maps[SM_EY], ea)) |
                (uint32_t)(map_apply(maps[SM_ER], ea + 1) * KP + map_apply(maps[SM_EY], ea + 1)) << 16;
    }
#pragma unroll
    for (int k = 0; k < CPT; k++) {
        const int ec = 2 * ((tid + 256 * k) & (hC - 1));
        oC[k] = (uint32_t)map_apply(maps[SM_EC], ec) * (WIDE ? 1u : 8u);
        sC[k] = (uint32_t)(map_apply(maps[SM_ER2], ec) * FP + map_apply(maps[SM_EF], ec)) |
                (uint32_t)(map_apply(maps[SM_ER2], ec + 1) * FP + map_apply(maps[SM_EF], ec + 1)) << 16;
    }
    // MFMA lane roles: A operand row `col`, k = 4t + g; B operand k = 4t + g,
    // column `col`; result rows 4g + v, column `col`
    const int g = lane >> 4, col = lane & 15, cpart = g & 1;
    const int wrow0 = wave * (R >> 2), rbw = R >> 6;
    float bq[NT][NC];
    int64_t bcur = -1;
    const int64_t n_tiles = (int64_t)1 << (nr - L);
    int64_t t = blockIdx.x;
    if (t >= n_tiles) return; // whole workgroup
    // two tiles of A in flight: the workgroup's next two tiles are loaded into
    // registers (pa0, pa1 in turn) while the current one is computed
    u32x4 pa0[4], pa1[4];
    const int64_t G = gridDim.x;
    auto load = [&](u32x4 (&pa)[4], int64_t tt) {
        if constexpr (WIDE) {
            const float2 *base = A + map_apply(maps[SM_RA], tt << L);
#pragma unroll
            for (int k = 0; k < 4; k++) pa[k] = *reinterpret_cast<const u32x4 *>(base + oA[k]);
        } else {
            const __amdgpu_buffer_rsrc_t r = tile_rsrc(A + map_apply(maps[SM_RA], tt << L));
#pragma unroll
            for (int k = 0; k < 4; k++) pa[k] = __builtin_amdgcn_raw_buffer_load_b128(r, oA[k], 0, 0);
        }
    };
    load(pa0, t);
    load(pa1, t + G < n_tiles ? t + G : t);
    // One tile: stage its prefetched A, load the A two tiles ahead into the
    // same registers, multiply, store C.  The loop is unrolled by two so that
    // the register sets alternate statically, and the wait before staging
    // covers only the loads of the set being staged.
    auto tile = [&](int64_t t, u32x4 (&pa)[4]) {
        const int64_t r0 = t << L;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            TA[sA[k] & 0xffffu] = make_float2(__uint_as_float(pa[k].x), __uint_as_float(pa[k].y));
            TA[sA[k] >> 16] = make_float2(__uint_as_float(pa[k].z), __uint_as_float(pa[k].w));
        }
        // the B matrix of this wave's rows, as the lane's entries of B'
        const int64_t bb = map_apply(maps[SM_RB], r0 + wrow0);
        if (bb != bcur) {
            bcur = bb;
#pragma unroll
            for (int s = 0; s < NT; s++) {
                const int y = 2 * s + (g >> 1);
#pragma unroll
                for (int cb = 0; cb < NC; cb++) {
                    const int jp = col + 16 * cb, f = jp >> 1, d = jp & 1;
                    float v = 0.f;
                    if (y < K && f < F) {
                        const float2 x = B[bb + map_apply(maps[SM_YB], y) + map_apply(maps[SM_FB], f)];
                        v = d == cpart ? x.x : (cpart ? -x.y : x.y);
                    }
                    bq[s][cb] = v;
                }
            }
            // settle these loads here, so that no later wait has to cover them
            __builtin_amdgcn_s_waitcnt(0x0f70); // vmcnt(0)
        }
        __syncthreads();
        // the A two tiles ahead (the current one again, an L2 hit, past the end)
        load(pa, t + 2 * G < n_tiles ? t + 2 * G : t);
        for (int q = 0; q < rbw; q++) {
            const int rb = wrow0 + 16 * q;
            floatx4 acc[NC];
#pragma unroll
            for (int cb = 0; cb < NC; cb++) acc[cb] = floatx4{0.f, 0.f, 0.f, 0.f};
            const float *arow = TAf + (rb + col) * RSA + g; // A[row][k' = 4s + g]
#pragma unroll
            for (int s = 0; s < NT; s++) {
                float a = 0.f;
                if (K >= 2 || (g >> 1) == 0) a = arow[4 * s];
#pragma unroll
                for (int cb = 0; cb < NC; cb++)
                    acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bq[s][cb], acc[cb], 0, 0, 0);
            }
#pragma unroll
            for (int cb = 0; cb < NC; cb++) {
                const int jp = col + 16 * cb, f = jp >> 1, d = jp & 1;
                if (f < F) {
#pragma unroll
                    for (int v = 0; v < 4; v++) TCf[2 * ((rb + 4 * g + v) * FP + f) + d] = acc[cb][v];
                }
            }
        }
        __syncthreads();
        if constexpr (WIDE) {
            float2 *cbase = C + map_apply(maps[SM_RC], r0);
#pragma unroll
            for (int k = 0; k < CPT; k++) {
                const float2 lo = TC[sC[k] & 0xffffu], hi = TC[sC[k] >> 16];
                const u32x4 v = {__float_as_uint(lo.x), __float_as_uint(lo.y), __float_as_uint(hi.x),
                                 __float_as_uint(hi.y)};
                *reinterpret_cast<u32x4 *>(cbase + oC[k]) = v;
            }
        } else {
            const __amdgpu_buffer_rsrc_t w = tile_rsrc(C + map_apply(maps[SM_RC], r0));
#pragma unroll
            for (int k = 0; k < CPT; k++) {
                const float2 lo = TC[sC[k] & 0xffffu], hi = TC[sC[k] >> 16];
                const u32x4 v = {__float_as_uint(lo.x), __float_as_uint(lo.y), __float_as_uint(hi.x),
                                 __float_as_uint(hi.y)};
                __builtin_amdgcn_raw_buffer_store_b128(v, w, oC[k], 0, 0);
            }
        }
    };
    for (;;) {
        tile(t, pa0);
        if ((t += G) >= n_tiles) break;
        tile(t, pa1);
        if ((t += G) >= n_tiles) break;
    }
}

// Long contraction on matrix cores: the same real block product as
// k_stream_mx, for 2^kc >= 64.  A workgroup owns 64 rows (16 per wave, one
// B matrix) and a range of 32-wide chunks of the contracted index.  Each chunk
// is staged through LDS while the next one is loaded into registers: A as
// floats ([row][2y + c], row stride 68, so that a wave's operand reads -- 16
// rows by 4 consecutive floats -- fall in 64 distinct banks) and B already in
// its real block form B'[2y + c][2f + d] (row stride SB = 16 mod 64, so that
// the 4 rows a read spans use disjoint banks), which makes every matrix-core
// operand one 32-bit LDS read.  With one chunk range per row group the
// outputs go straight to C (through LDS, coalesced); otherwise each range's
// partial sums go to P[split][r][f] and k_stream_lk_sum adds the ranges in
// order.
template <int NC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_stream_lk(const float2 *__restrict__ A, const float2 *__restrict__ B,
                                                   float2 *__restrict__ P, float2 *__restrict__ C,
                                                   const BitMap *__restrict__ maps, int nr, int kc, int nf, int ks) {
    constexpr int RS = 68, SB = NC == 1 ? 16 : 16 * NC + 16, NT = 16;
    __shared__ float TA[64 * RS];
    __shared__ float TB[64 * SB];
    const int F = 1 << nf, nBt = 32 << nf;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, col = lane & 15;
    const int nch = 1 << (kc - 5 - ks);
    // work items: (row group, chunk range) pairs, dealt to a persistent grid
    const int64_t n_items = (int64_t)1 << (nr - 6 + ks), G = gridDim.x;
    int64_t item = blockIdx.x;
    if (item >= n_items) return; // whole workgroup
    // A chunk elements: when the tile's lowest bit is A's lowest (the maps are
    // bit deposits, so then every element pair 2i, 2i + 1 is adjacent and 16-byte
    // aligned), a thread loads four such pairs with 16-byte loads; otherwise
    // eight single elements
    const bool pairs = map_apply(maps[SM_EA], 1) == 1;
    int offA[8], sA[8], offB[4], sB[4];
#pragma unroll
    for (int k = 0; k < 8; k++) {
        const int e = pairs ? 2 * (tid + 256 * (k >> 1)) + (k & 1) : tid + 256 * k;
        offA[k] = (int)map_apply(maps[SM_EA], e);
        sA[k] = (int)map_apply(maps[SM_ER], e) * RS + 2 * (int)map_apply(maps[SM_EY], e);
    }
    // B chunk elements with the new index f fastest across lanes: their two
    // 8-byte LDS writes per element then fall in consecutive banks (with the
    // chunk index y fastest, as in B's memory order, rows 2y SB apart hit two
    // banks only); B is small and read from L2, so its gather costs little
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int e = tid + 256 * k, f = e & (F - 1), yl = e >> nf;
        offB[k] = e < nBt ? (int)(map_apply(maps[SM_YB], yl) + map_apply(maps[SM_FB], f)) : 0;
        sB[k] = e < nBt ? 2 * yl * SB + 2 * f : 0;
    }
    // with one chunk range per row group: this thread's output elements of a
    // work item (C offset from the item's base, LDS source), the same for every
    // item, so the bit maps are evaluated once
    const int nC = 64 << nf, FP = F + 2;
    int offC[8], srcC[8];
#pragma unroll
    for (int k = 0; k < 8; k++) {
        const int e = tid + 256 * k;
        const bool on = ks == 0 && e < nC;
        offC[k] = on ? (int)map_apply(maps[SM_EC], e) : 0;
        srcC[k] = on ? (int)map_apply(maps[SM_ER2], e) * FP + (int)map_apply(maps[SM_EF], e) : 0;
    }
    // B' columns 2f + d with f >= F (fewer than 8 new indices) stay zero: the
    // stagings only write the others
    for (int i = tid; i < 64 * SB; i += 256) TB[i] = 0.f;
    // A and B offsets of each chunk's first contracted element, evaluated once
    // per workgroup (up to 64 chunks): a bit map costs a chain of dependent
    // scalar loads, which would otherwise sit before every chunk's loads
    __shared__ int64_t YT[2][64];
    const int n_ch = 1 << (kc - 5);
    const bool ytab = n_ch <= 64;
    if (ytab)
        for (int c = tid; c < n_ch; c += 256) {
            YT[0][c] = map_apply(maps[SM_YA], (int64_t)c << 5);
            YT[1][c] = map_apply(maps[SM_YB], (int64_t)c << 5);
        }
    __syncthreads();
    float2 pa[8], pb[4];
    auto load = [&](int64_t abase, int64_t bbase, int ch) {
        const int64_t ya = abase + (ytab ? YT[0][ch] : map_apply(maps[SM_YA], (int64_t)ch << 5));
        const int64_t yb = bbase + (ytab ? YT[1][ch] : map_apply(maps[SM_YB], (int64_t)ch << 5));
        if (pairs) {
#pragma unroll
            for (int k = 0; k < 8; k += 2) {
                const float4 v = *reinterpret_cast<const float4 *>(A + ya + offA[k]);
                pa[k] = make_float2(v.x, v.y);
                pa[k + 1] = make_float2(v.z, v.w);
            }
        } else {
#pragma unroll
            for (int k = 0; k < 8; k++) pa[k] = A[ya + offA[k]];
        }
#pragma unroll
        for (int k = 0; k < 4; k++)
            if (tid + 256 * k < nBt) pb[k] = B[yb + offB[k]];
    };
    // the row group and first chunk of a work item
    auto start = [&](int64_t it, int64_t &r0, int64_t &abase, int64_t &bbase, int &sp) {
        r0 = (it >> ks) << 6;
        sp = (int)(it & ((1 << ks) - 1));
        abase = map_apply(maps[SM_RA], r0);
        bbase = map_apply(maps[SM_RB], r0);
    };
    int64_t r0, abase, bbase;
    int sp;
    start(item, r0, abase, bbase, sp);
    load(abase, bbase, sp * nch);
    __syncthreads(); // the zero fill of B' before its first staging
    // this lane's operands: A[row][k' = 4s + g], B'[k' = 4s + g][col + 16 cb]
    const float *arow = TA + (16 * wave + col) * RS + g;
    const float *bcol = TB + g * SB + col;
    for (;;) {
        const int64_t next = item + G;
        int64_t nr0 = 0, nabase = 0, nbbase = 0;
        int nsp = 0;
        if (next < n_items) start(next, nr0, nabase, nbbase, nsp);
        floatx4 acc[NC];
#pragma unroll
        for (int cb = 0; cb < NC; cb++) acc[cb] = floatx4{0.f, 0.f, 0.f, 0.f};
        const int c0 = sp * nch;
        for (int ch = c0; ch < c0 + nch; ch++) {
#pragma unroll
            for (int k = 0; k < 8; k++) *reinterpret_cast<float2 *>(TA + sA[k]) = pa[k];
#pragma unroll
            for (int k = 0; k < 4; k++)
                if (tid + 256 * k < nBt) {
                    *reinterpret_cast<float2 *>(TB + sB[k]) = pb[k];
                    *reinterpret_cast<float2 *>(TB + sB[k] + SB) = make_float2(-pb[k].y, pb[k].x);
                }
            __syncthreads();
            // the next chunk, or the next work item's first chunk
            if (ch + 1 < c0 + nch) load(abase, bbase, ch + 1);
            else if (next < n_items) load(nabase, nbbase, nsp * nch);
            // operands of SG s-steps at a time, the next SG read from LDS
            // while these feed the matrix cores (two register slots)
            constexpr int SG = NC >= 4 ? 2 : 4;
            float av[2][SG], bv[2][SG][NC];
            auto lds_ops = [&](int sl, int s0) {
#pragma unroll
                for (int q = 0; q < SG; q++) {
                    av[sl][q] = arow[4 * (s0 + q)];
#pragma unroll
                    for (int cb = 0; cb < NC; cb++) bv[sl][q][cb] = bcol[4 * (s0 + q) * SB + 16 * cb];
                }
            };
            lds_ops(0, 0);
#pragma unroll
            for (int sg = 0; sg < NT / SG; sg++) {
                const int sl = sg & 1;
                if (sg + 1 < NT / SG) lds_ops(sl ^ 1, SG * (sg + 1));
                __builtin_amdgcn_sched_barrier(0); // keep those reads ahead of these products
#pragma unroll
                for (int q = 0; q < SG; q++)
#pragma unroll
                    for (int cb = 0; cb < NC; cb++)
                        acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[sl][q], bv[sl][q][cb], acc[cb], 0, 0, 0);
            }
            __syncthreads();
        }
        if (ks == 0) {
            // one chunk range: the 64 x F outputs go to C through LDS ([row][f],
            // row stride F+2, in TA's space), written in C's memory order
#pragma unroll
            for (int cb = 0; cb < NC; cb++) {
                const int jp = col + 16 * cb, f = jp >> 1, d = jp & 1;
                if (f < F) {
#pragma unroll
                    for (int v = 0; v < 4; v++) TA[2 * ((16 * wave + 4 * g + v) * FP + f) + d] = acc[cb][v];
                }
            }
            __syncthreads();
            const float2 *TC = reinterpret_cast<const float2 *>(TA);
            float2 *cb = C + map_apply(maps[SM_RC], r0);
#pragma unroll
            for (int k = 0; k < 8; k++)
                if (tid + 256 * k < nC) cb[offC[k]] = TC[srcC[k]];
            __syncthreads(); // TA is staged again by the next work item
        } else {
            float *Pf = reinterpret_cast<float *>(P);
            const int64_t pbase = ((int64_t)sp << (nr + nf)) + ((r0 + 16 * wave + 4 * g) << nf);
#pragma unroll
            for (int cb = 0; cb < NC; cb++) {
                const int jp = col + 16 * cb, f = jp >> 1, d = jp & 1;
                if (f < F) {
#pragma unroll
                    for (int v = 0; v < 4; v++) Pf[2 * (pbase + ((int64_t)v << nf) + f) + d] = acc[cb][v];
                }
            }
        }
        if (next >= n_items) break;
        item = next;
        r0 = nr0;
        abase = nabase;
        bbase = nbbase;
        sp = nsp;
    }
}

__global__ void __launch_bounds__(256) k_stream_lk_sum(const float2 *__restrict__ P, float2 *__restrict__ C,
                                                       const BitMap *__restrict__ maps, int nr, int nf, int ks) {
    const int64_t n = (int64_t)1 << (nr + nf);
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        float2 s = P[i];
        for (int j = 1; j < (1 << ks); j++) {
            const float2 x = P[((int64_t)j << (nr + nf)) + i];
            s.x += x.x;
            s.y += x.y;
        }
        C[map_apply(maps[SM_RC], i >> nf) + map_apply(maps[SM_FC], i & ((1 << nf) - 1))] = s;
    }
}

// Fused pair of streaming contractions on matrix cores, C2 = (A1 B1) B2 with
// the intermediate kept in LDS (the tile legs are described with StreamOp).
// Stage 1 is the k_stream_mx tile with 64 rows, 2^KC1 contracted and
// F1 = 8 NC1 new (16 or 32; one 16-row block per wave, the wave's B1' in
// registers); its 64 x F1 result goes to LDS as [row][f1] at a row stride of
// 36 complex.  Stage 2 reads that as 4 F1 rows r' = (row bits 0-1, f1) by 16
// contracted y2 = row bits 2-5 -- the stride makes a wave's operand reads (16
// rows by 4 floats) hit 64 distinct banks -- each wave F1 / 16 row blocks of
// 16 against B2' (registers; B2 depends only on outer row bits), 16 new legs.
// Its 4 F1 x 16 result is staged through the same LDS space ([r'][f2], row
// stride 18) and stored to C2 with 16-byte stores.  The next tile's A1 is
// loaded while a tile is computed.
template <int KC1, int NC1>
__global__ void __launch_bounds__(256) k_stream_mx2(const float2 *__restrict__ A, const float2 *__restrict__ B,
                                                    const float2 *__restrict__ B2, float2 *__restrict__ C,
                                                    const BitMap *__restrict__ maps, int nr) {
    constexpr int K1 = 1 << KC1, RSA = 2 * K1 + 4, KP = RSA / 2, NT1 = K1 / 2, FP1 = 36;
    constexpr int NT2 = 8, NC2 = 2, FP2 = 18, QB = NC1 / 2; // QB: stage-2 row blocks per wave
    __shared__ float2 TA[64 * KP];
    __shared__ float2 TC[64 * FP1]; // intermediate [64][FP1]; then the output [128][FP2]
    const float *TAf = reinterpret_cast<const float *>(TA);
    float *TCf = reinterpret_cast<float *>(TC);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, col = lane & 15, cpart = g & 1;
    // 16-byte moves of element pairs (tile bit 0 is tensor bit 0): A1's
    // 2^(6+KC1) elements (the pair index wraps for KC1 = 4) and C2's
    // 2^(9 + log2 NC1), NC1 pairs per thread
    constexpr int hA = (64 << KC1) >> 1;
    uint32_t oA[4], sA[4], oC[NC1], sC[NC1];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int ea = 2 * ((tid + 256 * k) & (hA - 1));
        oA[k] = (uint32_t)map_apply(maps[SM_EA], ea) * 8u;
        sA[k] = (uint32_t)(map_apply(maps[SM_ER], ea) * KP + map_apply(maps[SM_EY], ea)) |
                (uint32_t)(map_apply(maps[SM_ER], ea + 1) * KP + map_apply(maps[SM_EY], ea + 1)) << 16;
    }
#pragma unroll
    for (int k = 0; k < NC1; k++) {
        const int ec = 2 * (tid + 256 * k);
        oC[k] = (uint32_t)map_apply(maps[SM_EC], ec) * 8u;
        sC[k] = (uint32_t)(map_apply(maps[SM_ER2], ec) * FP2 + map_apply(maps[SM_EF], ec)) |
                (uint32_t)(map_apply(maps[SM_ER2], ec + 1) * FP2 + map_apply(maps[SM_EF], ec + 1)) << 16;
    }
    float bq1[NT1][NC1], bq2[NT2][NC2];
    int64_t bcur1 = -1, bcur2 = -1;
    const int64_t n_tiles = (int64_t)1 << (nr - 6), G = gridDim.x;
    int64_t t = blockIdx.x;
    if (t >= n_tiles) return; // whole workgroup
    u32x4 pa[4];
    auto load = [&](int64_t tt) {
        const __amdgpu_buffer_rsrc_t r = tile_rsrc(A + map_apply(maps[SM_RA], tt << 6));
#pragma unroll
        for (int k = 0; k < 4; k++) pa[k] = __builtin_amdgcn_raw_buffer_load_b128(r, oA[k], 0, 0);
    };
    load(t);
    for (;;) {
        const int64_t r0 = t << 6;
#pragma unroll
        for (int k = 0; k < 4; k++) {
            TA[sA[k] & 0xffffu] = make_float2(__uint_as_float(pa[k].x), __uint_as_float(pa[k].y));
            TA[sA[k] >> 16] = make_float2(__uint_as_float(pa[k].z), __uint_as_float(pa[k].w));
        }
        // B1 of this wave's rows and B2 of the tile, as the lanes' entries of
        // the real block forms
        const int64_t bb1 = map_apply(maps[SM_RB], r0 + 16 * wave), bb2 = map_apply(maps[SM_RB2], r0);
        if (bb1 != bcur1 || bb2 != bcur2) {
            bcur1 = bb1, bcur2 = bb2;
#pragma unroll
            for (int s = 0; s < NT1; s++) {
                const int y = 2 * s + (g >> 1);
#pragma unroll
                for (int cb = 0; cb < NC1; cb++) {
                    const int jp = col + 16 * cb, f = jp >> 1, d = jp & 1;
                    const float2 x = B[bb1 + map_apply(maps[SM_YB], y) + map_apply(maps[SM_FB], f)];
                    bq1[s][cb] = d == cpart ? x.x : (cpart ? -x.y : x.y);
                }
            }
#pragma unroll
            for (int s = 0; s < NT2; s++) {
                const int y = 2 * s + (g >> 1);
#pragma unroll
                for (int cb = 0; cb < NC2; cb++) {
                    const int jp = col + 16 * cb, f = jp >> 1, d = jp & 1;
                    const float2 x = B2[bb2 + map_apply(maps[SM_YB2], y) + map_apply(maps[SM_FB2], f)];
                    bq2[s][cb] = d == cpart ? x.x : (cpart ? -x.y : x.y);
                }
            }
            __builtin_amdgcn_s_waitcnt(0x0f70); // vmcnt(0): settle these loads here
        }
        __syncthreads();
        const int64_t tn = t + G;
        load(tn < n_tiles ? tn : t); // the next tile's A1 (the current one again at the end)
        // stage 1: this wave's 16 rows by F1 new, into the intermediate
        {
            floatx4 acc[NC1];
#pragma unroll
            for (int cb = 0; cb < NC1; cb++) acc[cb] = floatx4{0.f, 0.f, 0.f, 0.f};
            const int rb = 16 * wave;
            const float *arow = TAf + (rb + col) * RSA + g; // A1[row][k' = 4s + g]
#pragma unroll
            for (int s = 0; s < NT1; s++) {
                const float a = arow[4 * s];
#pragma unroll
                for (int cb = 0; cb < NC1; cb++)
                    acc[cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bq1[s][cb], acc[cb], 0, 0, 0);
            }
#pragma unroll
            for (int cb = 0; cb < NC1; cb++) {
                const int jp = col + 16 * cb, f = jp >> 1, d = jp & 1;
#pragma unroll
                for (int v = 0; v < 4; v++) TCf[2 * ((rb + 4 * g + v) * FP1 + f) + d] = acc[cb][v];
            }
        }
        __syncthreads();
        // stage 2: rows r' = 16 (QB wave + q) + col; operand (r', y2 = 2s + g/2,
        // part g%2) is intermediate row (r' & 3) | y2 << 2, column r' >> 2
        floatx4 acc2[QB][NC2];
#pragma unroll
        for (int q = 0; q < QB; q++) {
#pragma unroll
            for (int cb = 0; cb < NC2; cb++) acc2[q][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
            const int rp = 16 * (QB * wave + q) + col;
            const float *arow = TCf + 2 * ((rp & 3) * FP1 + (rp >> 2)) + 8 * FP1 * (g >> 1) + cpart;
#pragma unroll
            for (int s = 0; s < NT2; s++) {
                const float a = arow[16 * FP1 * s];
#pragma unroll
                for (int cb = 0; cb < NC2; cb++)
                    acc2[q][cb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, bq2[s][cb], acc2[q][cb], 0, 0, 0);
            }
        }
        __syncthreads(); // every read of the intermediate is done
#pragma unroll
        for (int q = 0; q < QB; q++) {
            const int rb = 16 * (QB * wave + q);
#pragma unroll
            for (int cb = 0; cb < NC2; cb++) {
                const int jp = col + 16 * cb, f = jp >> 1, d = jp & 1;
#pragma unroll
                for (int v = 0; v < 4; v++) TCf[2 * ((rb + 4 * g + v) * FP2 + f) + d] = acc2[q][cb][v];
            }
        }
        __syncthreads();
        const __amdgpu_buffer_rsrc_t w = tile_rsrc(C + map_apply(maps[SM_RC], r0));
#pragma unroll
        for (int k = 0; k < NC1; k++) {
            const float2 lo = TC[sC[k] & 0xffffu], hi = TC[sC[k] >> 16];
            const u32x4 v = {__float_as_uint(lo.x), __float_as_uint(lo.y), __float_as_uint(hi.x), __float_as_uint(hi.y)};
            __builtin_amdgcn_raw_buffer_store_b128(v, w, oC[k], 0, 0);
        }
        if ((t = tn) >= n_tiles) break;
    }
}

// Workgroups of `fn` (256 threads, `lds` bytes of dynamic LDS) that the
// current device holds at once; persistent grids are sized to this so that no
// workgroup waits for another to finish before it starts.
static int64_t resident_blocks(const void *fn, size_t lds) {
    static std::mutex mu;
    static std::map<std::tuple<int, const void *, size_t>, int64_t> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) fail(RQC_EDEVICE, "hipGetDevice failed");
    std::lock_guard<std::mutex> lock(mu);
    const auto key = std::make_tuple(dev, fn, lds);
    const auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds) != hipSuccess || per_cu < 1) per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
    return cache[key] = (int64_t)per_cu * cus;
}

template <int KC, int NC, bool WIDE>
void launch_stream_mx_wide(const StreamOp &op, const BitMap *d_maps, const float2 *a, const float2 *b, float2 *c,
                           hipStream_t s) {
    const int L = op.tile_l;
    const int rsa = ((1 << KC) >= 4 ? 2 * (1 << KC) : 8) + 4; // floats per A row, as in the kernel
    const size_t lds = sizeof(float2) * (((size_t)1 << L) * (rsa / 2) + ((size_t)1 << L) * ((1 << op.nf) + 2));
    const int64_t tiles = (int64_t)1 << (op.nr - L);
    const int64_t res = resident_blocks(reinterpret_cast<const void *>(&k_stream_mx<KC, NC, WIDE>), lds);
    const dim3 g((unsigned)std::min<int64_t>(tiles, res)), t(256);
    hipLaunchKernelGGL((k_stream_mx<KC, NC, WIDE>), g, t, lds, s, a, b, c, d_maps, op.nr, op.nf, L);
}

template <int KC, int NC>
void launch_stream_mx_nc(const StreamOp &op, const BitMap *d_maps, const float2 *a, const float2 *b, float2 *c,
                         hipStream_t s) {
    if (op.wide) launch_stream_mx_wide<KC, NC, true>(op, d_maps, a, b, c, s);
    else launch_stream_mx_wide<KC, NC, false>(op, d_maps, a, b, c, s);
}

template <int KC>
void launch_stream_mx(const StreamOp &op, const BitMap *d_maps, const float2 *a, const float2 *b, float2 *c,
                      hipStream_t s) {
    if (op.nf <= 3) launch_stream_mx_nc<KC, 1>(op, d_maps, a, b, c, s);
    else if (op.nf == 4) launch_stream_mx_nc<KC, 2>(op, d_maps, a, b, c, s);
    else if (op.nf == 5) launch_stream_mx_nc<KC, 4>(op, d_maps, a, b, c, s);
    else launch_stream_mx_nc<KC, 8>(op, d_maps, a, b, c, s);
}

void launch_stream(const StreamOp &op, const BitMap *d_maps, const float2 *a, const float2 *b, float2 *c,
                   float2 *w, const float2 *b2, hipStream_t s) {
    const int kind = stream_kernel(op);
    if (kind == SK_MX2) {
        if (op.tile_l != 6 || (op.kc != 4 && op.kc != 5) || op.nf != 5 || op.kc2 != 4 || op.nf2 != 4 || op.nr < 8 ||
            op.nr > 36 || !b2)
            fail(RQC_EPLAN, "fused streaming pair exceeds the kernel's limits");
        const int64_t tiles = (int64_t)1 << (op.nr - 6);
        auto go = [&](auto kern) {
            const int64_t res = resident_blocks(reinterpret_cast<const void *>(kern), 0);
            hipLaunchKernelGGL(kern, dim3((unsigned)std::min<int64_t>(tiles, res)), dim3(256), 0, s, a, b, b2, c,
                               d_maps, op.nr);
        };
        if (op.kc == 4) go(k_stream_mx2<4, 4>);
        else go(k_stream_mx2<5, 4>);
        return;
    }
    if (kind == SK_MX) {
        if (op.tile_l < 6 || op.tile_l > 8 || op.tile_l + op.kc > 11 || op.tile_l + op.nf > (op.nf == 6 ? 12 : 11) ||
            op.kc > 5 || op.nf > 6 || op.nr < op.tile_l)
            fail(RQC_EPLAN, "matrix-core streaming tile exceeds the kernel's limits");
        switch (op.kc) {
        case 0: launch_stream_mx<0>(op, d_maps, a, b, c, s); break;
        case 1: launch_stream_mx<1>(op, d_maps, a, b, c, s); break;
        case 2: launch_stream_mx<2>(op, d_maps, a, b, c, s); break;
        case 3: launch_stream_mx<3>(op, d_maps, a, b, c, s); break;
        case 4: launch_stream_mx<4>(op, d_maps, a, b, c, s); break;
        default: launch_stream_mx<5>(op, d_maps, a, b, c, s); break;
        }
        return;
    }
    if (kind == SK_LK) {
        if (op.kc < 6 || op.nf > 5 || op.nr < 6 || op.lk_split < 0 || op.lk_split > op.kc - 5 || (op.lk_split && !w))
            fail(RQC_EPLAN, "long streaming contraction exceeds the kernel's limits");
        const int64_t items = (int64_t)1 << (op.nr - 6 + op.lk_split);
        auto go = [&](auto kern) {
            // persistent grid: the per-workgroup set-up (offset tables, B' zero
            // columns) is paid once per resident workgroup, not per row group
            const int64_t res = resident_blocks(reinterpret_cast<const void *>(kern), 0);
            hipLaunchKernelGGL(kern, dim3((unsigned)std::min<int64_t>(items, res)), dim3(256), 0, s, a, b, w, c,
                               d_maps, op.nr, op.kc, op.nf, op.lk_split);
        };
        if (op.nf <= 3) go(k_stream_lk<1>);
        else if (op.nf == 4) go(k_stream_lk<2>);
        else go(k_stream_lk<4>);
        const dim3 t(256);
        if (op.lk_split > 0) {
            const int64_t n = (int64_t)1 << (op.nr + op.nf);
            const dim3 g2((unsigned)std::min<int64_t>((n + 255) / 256, 256 * 16));
            hipLaunchKernelGGL(k_stream_lk_sum, g2, t, 0, s, w, c, d_maps, op.nr, op.nf, op.lk_split);
        }
        return;
    }
    if (kind == SK_KY) {
        const int64_t waves = (int64_t)1 << op.nr;
        const dim3 g((unsigned)((waves + 3) / 4)), t(256);
        hipLaunchKernelGGL((k_stream_ky<16>), g, t, 0, s, a, b, c, d_maps, op.nr, op.kc, op.nf);
        return;
    }
    if (kind == SK_TILE) {
        if (op.tile_l > 8 || op.tile_l + op.kc > 11 || op.tile_l + op.nf > 11 || op.kc > 5)
            fail(RQC_EPLAN, "streaming tile exceeds the kernel's limits");
        const int64_t tiles = (int64_t)1 << (op.nr - op.tile_l);
        const dim3 g((unsigned)std::min<int64_t>(tiles, 256 * 8)), t(256);
        if (op.kc <= 3 && op.nf <= 3)
            hipLaunchKernelGGL((k_stream_tile<8, 8>), g, t, 0, s, a, b, c, d_maps, op.nr, op.kc, op.nf, op.tile_l);
        else if (op.nf <= 3)
            hipLaunchKernelGGL((k_stream_tile<32, 8>), g, t, 0, s, a, b, c, d_maps, op.nr, op.kc, op.nf, op.tile_l);
        else
            hipLaunchKernelGGL((k_stream_tile<32, 0>), g, t, 0, s, a, b, c, d_maps, op.nr, op.kc, op.nf, op.tile_l);
        return;
    }
    // SK_GEN
    const int64_t n = (int64_t)1 << op.rc;
    const unsigned gb = (unsigned)std::min<int64_t>((n + 255) / 256, 256 * 64);
    hipLaunchKernelGGL(k_stream_gen, dim3(gb), dim3(256), 0, s, a, b, c, d_maps, op.nr, op.kc, op.nf);
}

// ------------------------------------------------------------------ permute
PermDesc make_perm_desc(int r, const std::vector<int> &perm) {
    PermDesc d;
    // tile = the low 5 source bits, the source bits of the low 5 destination
    // bits, then more low source bits up to 2^10 elements
    const int t = r < 5 ? r : 5;
    std::vector<char> inT(r, 0);
    for (int i = 0; i < t; i++) inT[i] = 1;
    for (int i = 0; i < r; i++)
        if (perm[i] < t) inT[i] = 1;
    int cnt = 0;
    for (int i = 0; i < r; i++) cnt += inT[i];
    for (int i = 0; i < r && cnt < 10; i++)
        if (!inT[i]) inT[i] = 1, cnt++;
    std::vector<int> T, tb;
    for (int i = 0; i < r; i++) (inT[i] ? T : tb).push_back(i);
    d.tile_log = (int)T.size();
    d.n_tiles = (int64_t)1 << tb.size();
    std::vector<int> m1(tb.size()), m2(tb.size());
    for (size_t j = 0; j < tb.size(); j++) m1[j] = tb[j], m2[j] = perm[tb[j]];
    d.tile_src = make_map(m1);
    d.tile_dst = make_map(m2);
    std::vector<int> rd(T.size());
    for (size_t j = 0; j < T.size(); j++) rd[j] = T[j];
    d.rd = make_map(rd);
    std::vector<int> W(T.size());
    for (size_t j = 0; j < T.size(); j++) W[j] = (int)j; // positions in T
    std::sort(W.begin(), W.end(), [&](int x, int y) { return perm[T[x]] < perm[T[y]]; });
    std::vector<int> wl(T.size()), wd(T.size());
    for (size_t j = 0; j < T.size(); j++) wl[j] = W[j], wd[j] = perm[T[W[j]]];
    d.wr_lds = make_map(wl);
    d.wr_dst = make_map(wd);
    return d;
}

// One tile (at most 1024 elements) per iteration: read in source order
// (coalesced on the low source bits), write in destination order (coalesced on
// the low destination bits) through a padded LDS tile.
__device__ __forceinline__ void permute_tiles(const PermDesc &d, const float2 *__restrict__ src,
                                              float2 *__restrict__ dst, float2 *tile) {
    const int n = 1 << d.tile_log;
    const int tid = threadIdx.x;
    int64_t rd[4], wd[4];
    int wl[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
        const int i = tid + 256 * k;
        rd[k] = i < n ? map_apply(d.rd, i) : 0;
        wd[k] = i < n ? map_apply(d.wr_dst, i) : 0;
        const int l = i < n ? (int)map_apply(d.wr_lds, i) : 0;
        wl[k] = l + (l >> 5);
    }
    for (int64_t t = blockIdx.x; t < d.n_tiles; t += gridDim.x) {
        const int64_t bs = map_apply(d.tile_src, t), bd = map_apply(d.tile_dst, t);
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int i = tid + 256 * k;
            if (i < n) tile[i + (i >> 5)] = src[bs + rd[k]];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 4; k++) {
            const int i = tid + 256 * k;
            if (i < n) dst[bd + wd[k]] = tile[wl[k]];
        }
        __syncthreads();
    }
}

// descriptor in device memory (plans upload theirs once)
__global__ void __launch_bounds__(256) k_permute(const PermDesc *__restrict__ dp, const float2 *__restrict__ src,
                                                 float2 *__restrict__ dst) {
    __shared__ float2 tile[1024 + 32];
    permute_tiles(*dp, src, dst, tile);
}

// descriptor passed by value in the kernel arguments (no device copy needed)
__global__ void __launch_bounds__(256) k_permute_v(const PermDesc d, const float2 *__restrict__ src,
                                                   float2 *__restrict__ dst) {
    __shared__ float2 tile[1024 + 32];
    permute_tiles(d, src, dst, tile);
}

static unsigned permute_blocks(int64_t n_tiles) { return (unsigned)std::min<int64_t>(n_tiles, 256 * 32); }

void launch_permute(const PermDesc *d_desc, int64_t n_tiles, const float2 *src, float2 *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_permute, dim3(permute_blocks(n_tiles)), dim3(256), 0, s, d_desc, src, dst);
}

void launch_permute_value(const PermDesc &d, const float2 *src, float2 *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_permute_v, dim3(permute_blocks(d.n_tiles)), dim3(256), 0, s, d, src, dst);
}

// ------------------------------------------------------------------ complex GEMM, FP32 MFMA
// Offset of C element (m, n) within one batch: [m][n], or with the t = ins_bits
// low bits of m placed between bits s - 1 and s of n (s = ins_pos), for a
// consumer whose tiles want those M legs among C's lowest positions.
__device__ __forceinline__ int64_t gemm_c_off(int64_t m, int64_t n, int64_t N, int s, int t) {
    if (t == 0) return m * N + n;
    const int64_t lo_n = n & ((1LL << s) - 1), lo_m = m & ((1LL << t) - 1);
    return lo_n | (lo_m << s) | ((n >> s) << (s + t)) | ((m >> t) * (N << t));
}

typedef float floatx16 __attribute__((ext_vector_type(16)));

// Block tile BM x BN complex outputs, BK complex k per stage, 4 waves in a
// 2 x 2 grid, each wave (BM/2) x (BN/2) as 32 x 32 MFMA blocks.  Operands are
// staged de-interleaved (separate re / im planes) in LDS, double buffered.
// The complex product takes three real products (Gauss):
//   T1 = A_re B_re, T2 = A_im B_im, T3 = (A_re + A_im)(B_re + B_im),
//   C_re = T1 - T2, C_im = T3 - T1 - T2,
// three matrix-core products per complex multiply-add instead of four (the
// FP32 rounding error grows by about half: T3's terms are up to twice as large).
// waves per SIMD the registers are held to: the three accumulator sets take
// 3 * 16 * (BM / 64) * (BN / 64) registers per lane
constexpr int gemm_waves(int BM, int BN) { return BM * BN > 8192 ? 2 : BM * BN > 4096 ? 3 : 4; }

// INS: C takes the bit-inserted layout (gemm_c_off); a separate instance, so
// that the plain [m][n] epilogue keeps its registers (the inserted form's
// addresses made the 128 x 128 instance spill, about 10 % of a K = 64 GEMM)
template <int BM, int BN, int A_KFAST, int B_NFAST, bool INS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(gemm_waves(BM, BN))))
k_cgemm_f32(GemmArgs g) {
    constexpr int BK = 8;
    constexpr int PAD = 4;
    constexpr int WM = BM / 64, WN = BN / 64; // 32x32 blocks per wave
    constexpr int EA = BM * BK / 256, EB = BN * BK / 256; // complex per thread per stage
    __shared__ float As[2][2][BK][BM + PAD];
    __shared__ float Bs[2][2][BK][BN + PAD];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t ntn = g.N / BN, ntm = g.M / BM;
    // workgroups go round-robin over the 8 XCDs; give each XCD a contiguous
    // run of tiles, so that tiles sharing an operand panel share that XCD's L2
    const int64_t nblk = gridDim.x;
    const int64_t bid0 = (nblk & 7) == 0 ? (int64_t)(blockIdx.x & 7) * (nblk >> 3) + (blockIdx.x >> 3)
                                          : (int64_t)blockIdx.x;
    // with split K the grid is ksplit copies of the tile grid, one per K range
    const int64_t ntiles = ntn * ntm * g.batch;
    const int64_t bid = bid0 % ntiles, krange = bid0 / ntiles;
    const int64_t bz = bid / (ntn * ntm);
    // consecutive tiles share the larger operand's panel: m runs fastest when
    // B is the larger operand (N > M), n otherwise
    const int64_t m0 = (g.m_fast ? bid % ntm : (bid / ntn) % ntm) * BM;
    const int64_t n0 = (g.m_fast ? (bid / ntm) % ntn : bid % ntn) * BN;
    const float2 *A = g.A + bz * g.sa;
    const float2 *B = g.B + bz * g.sb;
    float2 *C = g.ksplit > 1 ? g.W + (krange * g.batch + bz) * g.M * g.N : g.C + bz * g.sc;
    const int64_t M = g.M, N = g.N, K = g.K;
    // partial sums of a K range go to W as [m][n]; the final C takes C's layout
    // (the launcher picks INS only when the GEMM writes C itself with inserted bits)
    const int ins_pos = INS ? g.c_ins_pos : 0, ins_bits = INS ? g.c_ins_bits : 0;

    // per-thread global coordinates of its operand chunk
    int a_r, a_c, b_r, b_c; // A: (m or k row, offset), B likewise
    if (A_KFAST) { a_r = tid / (BK / EA); a_c = (tid % (BK / EA)) * EA; }      // m, k
    else { a_r = tid / (BM / EA); a_c = (tid % (BM / EA)) * EA; }              // k, m
    if (B_NFAST) { b_r = tid / (BN / EB); b_c = (tid % (BN / EB)) * EB; }      // k, n
    else { b_r = tid / (BK / EB); b_c = (tid % (BK / EB)) * EB; }              // n, k

    float2 ra[EA], rb[EB];
    auto gload = [&](int64_t k0) {
        const float2 *pa = A_KFAST ? A + (m0 + a_r) * K + k0 + a_c : A + (k0 + a_r) * M + m0 + a_c;
        const float2 *pb = B_NFAST ? B + (k0 + b_r) * N + n0 + b_c : B + (n0 + b_r) * K + k0 + b_c;
#pragma unroll
        for (int e = 0; e < EA; e += 2) {
            float4 v = *reinterpret_cast<const float4 *>(pa + e);
            ra[e] = make_float2(v.x, v.y);
            ra[e + 1] = make_float2(v.z, v.w);
        }
#pragma unroll
        for (int e = 0; e < EB; e += 2) {
            float4 v = *reinterpret_cast<const float4 *>(pb + e);
            rb[e] = make_float2(v.x, v.y);
            rb[e + 1] = make_float2(v.z, v.w);
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int e = 0; e < EA; e++) {
            int kk = A_KFAST ? a_c + e : a_r, mm = A_KFAST ? a_r : a_c + e;
            As[buf][0][kk][mm] = ra[e].x;
            As[buf][1][kk][mm] = ra[e].y;
        }
#pragma unroll
        for (int e = 0; e < EB; e++) {
            int kk = B_NFAST ? b_r : b_c + e, nn = B_NFAST ? b_c + e : b_r;
            Bs[buf][0][kk][nn] = rb[e].x;
            Bs[buf][1][kk][nn] = rb[e].y;
        }
    };

    floatx16 t1[WM][WN], t2[WM][WN], t3[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; i++)
#pragma unroll
        for (int j = 0; j < WN; j++)
#pragma unroll
            for (int v = 0; v < 16; v++) t1[i][j][v] = 0.f, t2[i][j][v] = 0.f, t3[i][j][v] = 0.f;

    const int64_t kb = krange * (K / g.ksplit); // this workgroup's K range
    const int nk = (int)(K / g.ksplit / BK);
    gload(kb);
    sstore(0);
    __syncthreads();
    for (int kt = 0; kt < nk; kt++) {
        const int cur = kt & 1;
        if (kt + 1 < nk) gload(kb + (int64_t)(kt + 1) * BK);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 2) {
            const int kr = kk + (lane >> 5);
            float are[WM], aim[WM], asum[WM], bre[WN], bim[WN], bsum[WN];
#pragma unroll
            for (int i = 0; i < WM; i++) {
                const int mm = wm * (BM / 2) + i * 32 + (lane & 31);
                are[i] = As[cur][0][kr][mm];
                aim[i] = As[cur][1][kr][mm];
                asum[i] = are[i] + aim[i];
            }
#pragma unroll
            for (int j = 0; j < WN; j++) {
                const int nn = wn * (BN / 2) + j * 32 + (lane & 31);
                bre[j] = Bs[cur][0][kr][nn];
                bim[j] = Bs[cur][1][kr][nn];
                bsum[j] = bre[j] + bim[j];
            }
#pragma unroll
            for (int i = 0; i < WM; i++)
#pragma unroll
                for (int j = 0; j < WN; j++) {
                    t1[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(are[i], bre[j], t1[i][j], 0, 0, 0);
                    t2[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(aim[i], bim[j], t2[i][j], 0, 0, 0);
                    t3[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(asum[i], bsum[j], t3[i][j], 0, 0, 0);
                }
        }
        if (kt + 1 < nk) sstore(cur ^ 1);
        __syncthreads();
    }
    // epilogue: 32x32 accumulator, lane holds column lane%32 and rows
    // 8*(v/4) + 4*(lane/32) + v%4.  The plain [m][n] form is its own loop,
    // so that its addresses stay incremental.
    if constexpr (INS) {
#pragma unroll
        for (int i = 0; i < WM; i++)
#pragma unroll
            for (int j = 0; j < WN; j++)
#pragma unroll
                for (int v = 0; v < 16; v++) {
                    const int64_t m = m0 + wm * (BM / 2) + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                    const int64_t n = n0 + wn * (BN / 2) + j * 32 + (lane & 31);
                    const float x1 = t1[i][j][v], x2 = t2[i][j][v];
                    C[gemm_c_off(m, n, N, ins_pos, ins_bits)] = make_float2(x1 - x2, (t3[i][j][v] - x1) - x2);
                }
        return;
    }
#pragma unroll
    for (int i = 0; i < WM; i++)
#pragma unroll
        for (int j = 0; j < WN; j++)
#pragma unroll
            for (int v = 0; v < 16; v++) {
                const int64_t m = m0 + wm * (BM / 2) + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int64_t n = n0 + wn * (BN / 2) + j * 32 + (lane & 31);
                const float x1 = t1[i][j][v], x2 = t2[i][j][v];
                C[m * N + n] = make_float2(x1 - x2, (t3[i][j][v] - x1) - x2);
            }
}

// ------------------------------------------------------------------ split-precision complex GEMM
// Each FP32 operand value is written as x * s = hi + lo with hi, lo in bf16 or
// fp16 (s = 1 for bf16; a per-tensor power of two for fp16 that brings the
// tensor's largest magnitude into [2^14, 2^15)).  A real product is taken as
// hi*hi' + hi*lo' + lo*hi' (lo*lo' dropped), accumulated in FP32 on MFMA.  The
// complex product uses the interleaved real view A'[m][2k+c] = (re, im) and
//   B'_re[2k][n] = re, B'_re[2k+1][n] = -im;  B'_im[2k][n] = im, B'_im[2k+1][n] = re,
// so C_re = A' B'_re and C_im = A' B'_im are plain real GEMMs over 2K.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 half8 __attribute__((ext_vector_type(8)));

template <bool F16>
struct SplitT {
    using E = __bf16;
    using V8 = bf16x8;
    static __device__ __forceinline__ floatx16 mma(V8 a, V8 b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};
template <>
struct SplitT<true> {
    using E = _Float16;
    using V8 = half8;
    static __device__ __forceinline__ floatx16 mma(V8 a, V8 b, floatx16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};

// scale exponent for a tensor whose largest magnitude is amax (fp16 mode)
__device__ __forceinline__ int split_exp(float amax) {
    if (!(amax > 0.f) || !isfinite(amax)) return 0;
    int e = ilogbf(amax);
    int s = 14 - e;
    return s < -120 ? -120 : (s > 120 ? 120 : s);
}

// Pipelined: stages of 8 complex k (16 real k, one MFMA depth) are loaded
// into registers two stages ahead, split into hi / lo and written to the other
// of two LDS buffers while the current one feeds the MFMAs (one barrier per
// stage).  A and B are both staged interleaved (re, im) per k; the two B
// operands of the real products, (re, -im) and (im, re) pairs, are formed in
// registers from the staged pairs: a sign flip of the upper half-word, and a
// half-word swap, of each 32-bit word.
typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));

template <int BM, int BN, int A_KFAST, int B_NFAST, bool F16>
__global__ void __launch_bounds__(256) k_cgemm_split(GemmArgs g, const unsigned *__restrict__ amax) {
    using E = typename SplitT<F16>::E;
    using V8 = typename SplitT<F16>::V8;
    constexpr int BK = 8, LD = 2 * BK + 8;
    constexpr int WM = BM / 64, WN = BN / 64;
    constexpr int EA = BM * BK / 256, EB = BN * BK / 256; // complex per thread per stage
    __shared__ __attribute__((aligned(16))) E Ah[2][BM][LD];
    __shared__ __attribute__((aligned(16))) E Al[2][BM][LD];
    __shared__ __attribute__((aligned(16))) E Bh[2][BN][LD];
    __shared__ __attribute__((aligned(16))) E Bl[2][BN][LD];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int64_t ntn = g.N / BN, ntm = g.M / BM;
    // workgroups go round-robin over the 8 XCDs; give each XCD a contiguous
    // run of tiles, so that tiles sharing an operand panel share that XCD's L2
    const int64_t nblk = gridDim.x;
    const int64_t bid0 = (nblk & 7) == 0 ? (int64_t)(blockIdx.x & 7) * (nblk >> 3) + (blockIdx.x >> 3)
                                          : (int64_t)blockIdx.x;
    // with split K the grid is ksplit copies of the tile grid, one per K range
    const int64_t ntiles = ntn * ntm * g.batch;
    const int64_t bid = bid0 % ntiles, krange = bid0 / ntiles;
    const int64_t bz = bid / (ntn * ntm);
    // consecutive tiles share the larger operand's panel: m runs fastest when
    // B is the larger operand (N > M), n otherwise
    const int64_t m0 = (g.m_fast ? bid % ntm : (bid / ntn) % ntm) * BM;
    const int64_t n0 = (g.m_fast ? (bid / ntm) % ntn : bid % ntn) * BN;
    const float2 *A = g.A + bz * g.sa;
    const float2 *B = g.B + bz * g.sb;
    float2 *C = g.ksplit > 1 ? g.W + (krange * g.batch + bz) * g.M * g.N : g.C + bz * g.sc;
    const int64_t M = g.M, N = g.N, K = g.K;
    // partial sums of a K range go to W as [m][n]; the final C takes C's layout
    const int ins_pos = g.ksplit > 1 ? 0 : g.c_ins_pos, ins_bits = g.ksplit > 1 ? 0 : g.c_ins_bits;
    int ea = 0, eb = 0;
    if (F16) {
        ea = split_exp(__uint_as_float(amax[0]));
        eb = split_exp(__uint_as_float(amax[1]));
    }
    const float sa = ldexpf(1.f, ea), sb = ldexpf(1.f, eb);

    // per-thread operand chunk: EA (EB) complex values consecutive in memory
    int a_r, a_c, b_r, b_c;
    if (A_KFAST) { a_r = tid / (BK / EA); a_c = (tid % (BK / EA)) * EA; }      // m, k
    else { a_r = tid / (BM / EA); a_c = (tid % (BM / EA)) * EA; }              // k, m
    if (B_NFAST) { b_r = tid / (BN / EB); b_c = (tid % (BN / EB)) * EB; }      // k, n
    else { b_r = tid / (BK / EB); b_c = (tid % (BK / EB)) * EB; }              // n, k

    float4 ra[2][EA / 2], rb[2][EB / 2];
    auto gload = [&](int slot, int64_t k0) {
        const float2 *pa = A_KFAST ? A + (m0 + a_r) * K + k0 + a_c : A + (k0 + a_r) * M + m0 + a_c;
        const float2 *pb = B_NFAST ? B + (k0 + b_r) * N + n0 + b_c : B + (n0 + b_r) * K + k0 + b_c;
#pragma unroll
        for (int e = 0; e < EA / 2; e++) ra[slot][e] = *reinterpret_cast<const float4 *>(pa + 2 * e);
#pragma unroll
        for (int e = 0; e < EB / 2; e++) rb[slot][e] = *reinterpret_cast<const float4 *>(pb + 2 * e);
        // keep the loads here (a prefetch), not next to their use a stage later
        asm volatile("" ::: "memory");
    };
    auto sstore = [&](int slot, int buf) {
#pragma unroll
        for (int e = 0; e < EA; e++) {
            const float4 v = ra[slot][e >> 1];
            const float re = (e & 1 ? v.z : v.x) * sa, im = (e & 1 ? v.w : v.y) * sa;
            const E hr = (E)re, hi_ = (E)im;
            const E lr = (E)(re - (float)hr), li = (E)(im - (float)hi_);
            const int kk = A_KFAST ? a_c + e : a_r, mm = A_KFAST ? a_r : a_c + e;
            Ah[buf][mm][2 * kk] = hr;
            Ah[buf][mm][2 * kk + 1] = hi_;
            Al[buf][mm][2 * kk] = lr;
            Al[buf][mm][2 * kk + 1] = li;
        }
#pragma unroll
        for (int e = 0; e < EB; e++) {
            const float4 v = rb[slot][e >> 1];
            const float re = (e & 1 ? v.z : v.x) * sb, im = (e & 1 ? v.w : v.y) * sb;
            const E hr = (E)re, hi_ = (E)im;
            const E lr = (E)(re - (float)hr), li = (E)(im - (float)hi_);
            const int kk = B_NFAST ? b_r : b_c + e, nn = B_NFAST ? b_c + e : b_r;
            Bh[buf][nn][2 * kk] = hr;
            Bh[buf][nn][2 * kk + 1] = hi_;
            Bl[buf][nn][2 * kk] = lr;
            Bl[buf][nn][2 * kk + 1] = li;
        }
    };

    floatx16 cre[WM][WN], cim[WM][WN];
#pragma unroll
    for (int i = 0; i < WM; i++)
#pragma unroll
        for (int j = 0; j < WN; j++)
#pragma unroll
            for (int v = 0; v < 16; v++) cre[i][j][v] = 0.f, cim[i][j][v] = 0.f;

    const int ko = 8 * (lane >> 5);
    const u32x4v flip = {0x80000000u, 0x80000000u, 0x80000000u, 0x80000000u};
    auto compute = [&](int buf) {
        V8 ah[WM], al[WM], brh[WN], brl[WN], bih[WN], bil[WN];
#pragma unroll
        for (int i = 0; i < WM; i++) {
            const int mm = wm * (BM / 2) + i * 32 + (lane & 31);
            ah[i] = *reinterpret_cast<const V8 *>(&Ah[buf][mm][ko]);
            al[i] = *reinterpret_cast<const V8 *>(&Al[buf][mm][ko]);
        }
#pragma unroll
        for (int j = 0; j < WN; j++) {
            const int nn = wn * (BN / 2) + j * 32 + (lane & 31);
            const u32x4v h = __builtin_bit_cast(u32x4v, *reinterpret_cast<const V8 *>(&Bh[buf][nn][ko]));
            const u32x4v l = __builtin_bit_cast(u32x4v, *reinterpret_cast<const V8 *>(&Bl[buf][nn][ko]));
            brh[j] = __builtin_bit_cast(V8, h ^ flip);
            brl[j] = __builtin_bit_cast(V8, l ^ flip);
            bih[j] = __builtin_bit_cast(V8, (h >> 16) | (h << 16));
            bil[j] = __builtin_bit_cast(V8, (l >> 16) | (l << 16));
        }
#pragma unroll
        for (int i = 0; i < WM; i++)
#pragma unroll
            for (int j = 0; j < WN; j++) {
                cre[i][j] = SplitT<F16>::mma(ah[i], brh[j], cre[i][j]);
                cim[i][j] = SplitT<F16>::mma(ah[i], bih[j], cim[i][j]);
            }
#pragma unroll
        for (int i = 0; i < WM; i++)
#pragma unroll
            for (int j = 0; j < WN; j++) {
                cre[i][j] = SplitT<F16>::mma(ah[i], brl[j], cre[i][j]);
                cim[i][j] = SplitT<F16>::mma(ah[i], bil[j], cim[i][j]);
            }
#pragma unroll
        for (int i = 0; i < WM; i++)
#pragma unroll
            for (int j = 0; j < WN; j++) {
                cre[i][j] = SplitT<F16>::mma(al[i], brh[j], cre[i][j]);
                cim[i][j] = SplitT<F16>::mma(al[i], bih[j], cim[i][j]);
            }
    };

    // stage s lives in register slot s & 1 and LDS buffer s & 1; loads past
    // the last stage re-read it (unused), so that every iteration issues the
    // same loads and the waits before staging cover exactly one stage
    const int64_t kb = krange * (K / g.ksplit); // this workgroup's K range
    const int nk = (int)(K / g.ksplit / BK);
    gload(0, kb);
    gload(1, kb + (int64_t)std::min(1, nk - 1) * BK);
    sstore(0, 0);
    __syncthreads();
    // two stages per trip, so that register slots are compile-time indices
    auto stage = [&](auto par, int kt) {
        constexpr int cur = decltype(par)::value;
        gload(cur, kb + (int64_t)std::min(kt + 2, nk - 1) * BK); // stage kt is already in LDS
        compute(cur);
        if (kt + 1 < nk) sstore(cur ^ 1, cur ^ 1);
        __syncthreads();
    };
    for (int kt = 0; kt < nk; kt += 2) {
        stage(std::integral_constant<int, 0>{}, kt);
        if (kt + 1 < nk) stage(std::integral_constant<int, 1>{}, kt + 1);
    }
    // the plain [m][n] form is its own loop, so that its addresses stay incremental
    if (ins_bits) {
#pragma unroll
        for (int i = 0; i < WM; i++)
#pragma unroll
            for (int j = 0; j < WN; j++)
#pragma unroll
                for (int v = 0; v < 16; v++) {
                    const int64_t m = m0 + wm * (BM / 2) + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                    const int64_t n = n0 + wn * (BN / 2) + j * 32 + (lane & 31);
                    float re = cre[i][j][v], im = cim[i][j][v];
                    if (F16) {
                        re = ldexpf(ldexpf(re, -ea), -eb);
                        im = ldexpf(ldexpf(im, -ea), -eb);
                    }
                    C[gemm_c_off(m, n, N, ins_pos, ins_bits)] = make_float2(re, im);
                }
        return;
    }
#pragma unroll
    for (int i = 0; i < WM; i++)
#pragma unroll
        for (int j = 0; j < WN; j++)
#pragma unroll
            for (int v = 0; v < 16; v++) {
                const int64_t m = m0 + wm * (BM / 2) + i * 32 + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
                const int64_t n = n0 + wn * (BN / 2) + j * 32 + (lane & 31);
                float re = cre[i][j][v], im = cim[i][j][v];
                if (F16) {
                    re = ldexpf(ldexpf(re, -ea), -eb);
                    im = ldexpf(ldexpf(im, -ea), -eb);
                }
                C[m * N + n] = make_float2(re, im);
            }
}

__global__ void __launch_bounds__(256) k_absmax(const float *__restrict__ x, int64_t n, unsigned *__restrict__ out) {
    float m = 0.f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(x[i]));
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

__global__ void k_zero_u32(unsigned *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

template <int BM, int BN, bool F16>
static void split_dispatch(const GemmArgs &g, const unsigned *amax, hipStream_t s) {
    dim3 grid((unsigned)((g.N / BN) * (g.M / BM) * g.batch * g.ksplit));
    if (g.a_kfast && g.b_nfast) hipLaunchKernelGGL((k_cgemm_split<BM, BN, 1, 1, F16>), grid, dim3(256), 0, s, g, amax);
    else if (g.a_kfast) hipLaunchKernelGGL((k_cgemm_split<BM, BN, 1, 0, F16>), grid, dim3(256), 0, s, g, amax);
    else if (g.b_nfast) hipLaunchKernelGGL((k_cgemm_split<BM, BN, 0, 1, F16>), grid, dim3(256), 0, s, g, amax);
    else hipLaunchKernelGGL((k_cgemm_split<BM, BN, 0, 0, F16>), grid, dim3(256), 0, s, g, amax);
}

template <bool F16>
static void split_gemm(const GemmArgs &g, unsigned *amax, hipStream_t s) {
    if (F16) {
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, amax, 2);
        const int64_t na = 2 * g.batch * g.M * g.K, nb = 2 * g.batch * g.K * g.N;
        auto blocks = [](int64_t n) { return (unsigned)std::min<int64_t>((n + 255) / 256, 2048); };
        hipLaunchKernelGGL(k_absmax, dim3(blocks(na)), dim3(256), 0, s, (const float *)g.A, na, amax);
        hipLaunchKernelGGL(k_absmax, dim3(blocks(nb)), dim3(256), 0, s, (const float *)g.B, nb, amax + 1);
    }
    if (g.M >= 128 && g.N >= 128) split_dispatch<128, 128, F16>(g, amax, s);
    else if (g.M >= 128) split_dispatch<128, 64, F16>(g, amax, s);
    else if (g.N >= 128) split_dispatch<64, 128, F16>(g, amax, s);
    else split_dispatch<64, 64, F16>(g, amax, s);
}

template <int BM, int BN, bool INS>
static void gemm_dispatch_ins(const GemmArgs &g, hipStream_t s) {
    dim3 grid((unsigned)((g.N / BN) * (g.M / BM) * g.batch * g.ksplit));
    if (g.a_kfast && g.b_nfast) hipLaunchKernelGGL((k_cgemm_f32<BM, BN, 1, 1, INS>), grid, dim3(256), 0, s, g);
    else if (g.a_kfast) hipLaunchKernelGGL((k_cgemm_f32<BM, BN, 1, 0, INS>), grid, dim3(256), 0, s, g);
    else if (g.b_nfast) hipLaunchKernelGGL((k_cgemm_f32<BM, BN, 0, 1, INS>), grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((k_cgemm_f32<BM, BN, 0, 0, INS>), grid, dim3(256), 0, s, g);
}

template <int BM, int BN>
static void gemm_dispatch(const GemmArgs &g, hipStream_t s) {
    // with split K the tiles write partial sums as [m][n]; k_gemm_ksum inserts
    if (g.c_ins_bits > 0 && g.ksplit == 1) gemm_dispatch_ins<BM, BN, true>(g, s);
    else gemm_dispatch_ins<BM, BN, false>(g, s);
}

void launch_gemm_tiles(const GemmArgs &g, int precision, unsigned *amax, hipStream_t s);

// Split K: C = sum over ranges r (ascending) of W[r], one output per thread.
__global__ void __launch_bounds__(256) k_gemm_ksum(const float2 *__restrict__ W, float2 *__restrict__ C,
                                                   int64_t n, int64_t mn, int64_t sc, int ksplit, int64_t N,
                                                   int ins_pos, int ins_bits) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        float2 acc = W[i];
        for (int r = 1; r < ksplit; r++) {
            const float2 x = W[(int64_t)r * n + i];
            acc.x += x.x;
            acc.y += x.y;
        }
        const int64_t e = i % mn;
        C[(i / mn) * sc + gemm_c_off(e / N, e % N, N, ins_pos, ins_bits)] = acc;
    }
}

void launch_gemm(const GemmArgs &g_in, int precision, unsigned *amax, hipStream_t s) {
    GemmArgs g = g_in;
    g.m_fast = g.N > g.M;
    if (g.ksplit < 1 || (g.ksplit > 1 && (!g.W || g.K % (8LL * g.ksplit) != 0)))
        fail(RQC_EPLAN, "GEMM K split does not fit its kernel");
    if (g.c_ins_bits < 0 || g.c_ins_pos < 0 || (g.c_ins_bits > 0 && ((1LL << g.c_ins_pos) > g.N ||
                                                                     (1LL << g.c_ins_bits) > g.M)))
        fail(RQC_EPLAN, "GEMM output bit insertion does not fit its shape");
    launch_gemm_tiles(g, precision, amax, s);
    if (g.ksplit > 1) {
        const int64_t n = g.batch * g.M * g.N;
        hipLaunchKernelGGL(k_gemm_ksum, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 256 * 16)), dim3(256), 0, s,
                           g.W, g.C, n, g.M * g.N, g.sc, g.ksplit, g.N, g.c_ins_pos, g.c_ins_bits);
    }
}

void launch_gemm_tiles(const GemmArgs &g, int precision, unsigned *amax, hipStream_t s) {
    // the split kernels stage 16 complex k per step; shorter contractions stay FP32
    if (precision == RQC_BF16X3 && g.K >= 16) return split_gemm<false>(g, amax, s);
    if (precision == RQC_FP16X3 && g.K >= 16) return split_gemm<true>(g, amax, s);
    if (g.M >= 128 && g.N >= 128) gemm_dispatch<128, 128>(g, s);
    else if (g.M >= 128) gemm_dispatch<128, 64>(g, s);
    else if (g.N >= 128) gemm_dispatch<64, 128>(g, s);
    else gemm_dispatch<64, 64>(g, s);
}

// ------------------------------------------------------------------ FP64 accumulation
// acc[x] += sum over batched slices s (ascending) of root[open(x) + slice(s)],
// one add at a time in FP64, so the result does not depend on how slices are
// grouped into launches.
__global__ void __launch_bounds__(256) k_accumulate(const float2 *__restrict__ root, const BitMap *__restrict__ maps,
                                                    int64_t n, int64_t ns, double2 *__restrict__ acc) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int64_t ox = map_apply(maps[0], x);
    double2 a = acc[x];
    for (int64_t s = 0; s < ns; s++) {
        const float2 c = root[ox + map_apply(maps[1], s)];
        a.x += (double)c.x;
        a.y += (double)c.y;
    }
    acc[x] = a;
}

void launch_accumulate(const float2 *root, const BitMap *d_maps, int n_open, int n_batched, double2 *acc,
                       hipStream_t s) {
    const int64_t n = (int64_t)1 << n_open, ns = (int64_t)1 << n_batched;
    hipLaunchKernelGGL(k_accumulate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, root, d_maps, n, ns, acc);
}

__global__ void k_zero(double2 *p, int64_t n) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x < n) p[x] = make_double2(0.0, 0.0);
}

void launch_zero(double2 *acc, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, acc, n);
}

__global__ void k_finalize(const double2 *__restrict__ acc, int64_t n, double scale, float2 *__restrict__ out,
                           double2 *__restrict__ out64) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const double2 a = acc[x];
    const double re = a.x * scale, im = a.y * scale;
    out[x] = make_float2((float)re, (float)im);
    if (out64) out64[x] = make_double2(re, im);
}

void launch_finalize(const double2 *acc, int64_t n, double scale, float2 *out, double2 *out64, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, acc, n, scale, out, out64);
}

} // namespace rqc
