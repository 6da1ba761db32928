// Selection of the bitstrings with the largest probabilities in one open batch:
// step 4 of the linear-XEB spoofing recipe (Sec. III.B), which keeps the N
// entries of a batch B of 2^b amplitudes with the largest |amplitude|.
//
// p_t = (double)re^2 + (double)im^2 is the same on every route (each FP32
// square is exact in FP64, so the sum is rounded once, fused or not), and for
// p >= 0 the FP64 bit pattern orders like the value, so the selection is a
// radix select on 64-bit keys: six passes over the batch histogram one digit
// of the keys that still match the digits resolved so far (11, 11, 11, 11, 11
// and 8 bits below the sign), each followed by a one-workgroup pass that picks
// the digit holding the count-th largest key.  The result is the threshold key
// T and the number of entries equal to T still to take.  Ties at T go to the
// smallest batch indices, so the selected set is unique; it is written in
// ascending batch index by an ordered compaction (per-chunk counts, one scan
// workgroup, then each chunk writes its entries at its offset).
//
// All passes read the batch from HBM (8 bytes per entry per pass) and touch
// only a few KiB of scratch; the histogram is bounded by its 2048 bins.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace rqc {

namespace {

constexpr int kBins = 2048;
constexpr int kChunk = 4096; // entries per workgroup in the count and write passes
constexpr int kPasses = 6;
constexpr int kLo[kPasses] = {52, 41, 30, 19, 8, 0};
constexpr int kWidth[kPasses] = {11, 11, 11, 11, 11, 8};

struct SelState {
    uint64_t prefix;   // key digits resolved so far
    int64_t remaining; // entries still to take among those matching the prefix
};

__device__ __forceinline__ uint64_t key_of(float2 a) {
    const double re = (double)a.x, im = (double)a.y;
    return (uint64_t)__double_as_longlong(re * re + im * im);
}

__global__ void __launch_bounds__(256) k_sel_init(SelState *st, unsigned *hist, int64_t count) {
    for (int i = threadIdx.x; i < kBins; i += 256) hist[i] = 0;
    if (threadIdx.x == 0) {
        st->prefix = 0;
        st->remaining = count;
    }
}

// Histogram of the key digit [lo, lo + width) over the entries whose bits at
// and above lo + width equal the resolved prefix.
__global__ void __launch_bounds__(256) k_sel_hist(const float2 *__restrict__ amps, int64_t n, int lo, int width,
                                                  const SelState *__restrict__ st, unsigned *__restrict__ hist) {
    __shared__ unsigned h[kBins];
    for (int i = threadIdx.x; i < kBins; i += 256) h[i] = 0;
    __syncthreads();
    const uint64_t prefix = st->prefix;
    const int hi = lo + width;
    const uint64_t mask = (1ull << width) - 1;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const uint64_t k = key_of(amps[i]);
        if ((k >> hi) == prefix) atomicAdd(&h[(k >> lo) & mask], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kBins; i += 256)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

// One workgroup: the digit b whose bin holds the remaining-th largest key
// (counting from the top bin down); entries in higher bins are all taken.
// Clears the histogram for the next pass.
__global__ void __launch_bounds__(256) k_sel_pick(unsigned *__restrict__ hist, int width, SelState *__restrict__ st) {
    __shared__ int64_t suf[256];
    __shared__ unsigned bins[kBins];
    const int t = threadIdx.x;
    const int nb = 1 << width, per = nb / 256; // width >= 8
    int64_t s = 0;
    for (int j = 0; j < per; j++) {
        bins[t * per + j] = hist[t * per + j];
        s += bins[t * per + j];
    }
    suf[t] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) { // inclusive suffix sums
        const int64_t v = t + off < 256 ? suf[t + off] : 0;
        __syncthreads();
        suf[t] += v;
        __syncthreads();
    }
    const int64_t need = st->remaining;
    const int64_t above_t = t + 1 < 256 ? suf[t + 1] : 0;
    __syncthreads();
    if (suf[t] >= need && above_t < need) {
        int64_t above = above_t;
        int b = t * per + per - 1;
        for (; b > t * per; b--) {
            if (above + bins[b] >= need) break;
            above += bins[b];
        }
        st->remaining = need - above;
        st->prefix = (st->prefix << width) | (uint64_t)b;
    }
    for (int j = 0; j < per; j++) hist[t * per + j] = 0;
}

// Per chunk: entries above the threshold key T and entries equal to it.
__global__ void __launch_bounds__(256) k_sel_count(const float2 *__restrict__ amps, int64_t n,
                                                   const SelState *__restrict__ st, int2 *__restrict__ cnt) {
    __shared__ int red[2][4];
    const uint64_t T = st->prefix;
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    int gt = 0, eq = 0;
    for (int j = 0; j < kChunk / 256; j++) {
        const int64_t i = base + j * 256 + threadIdx.x;
        if (i < n) {
            const uint64_t k = key_of(amps[i]);
            gt += k > T;
            eq += k == T;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        gt += __shfl_down(gt, off, 64);
        eq += __shfl_down(eq, off, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[0][w] = gt, red[1][w] = eq;
    __syncthreads();
    if (threadIdx.x == 0)
        cnt[blockIdx.x] = make_int2(red[0][0] + red[0][1] + red[0][2] + red[0][3],
                                    red[1][0] + red[1][1] + red[1][2] + red[1][3]);
}

__device__ __forceinline__ int64_t imin(int64_t a, int64_t b) { return a < b ? a : b; }
__device__ __forceinline__ int64_t imax(int64_t a, int64_t b) { return a > b ? a : b; }

// Exclusive scan over 1024 per-thread totals in LDS.
__device__ int64_t block_exclusive_scan(int64_t v, int64_t *buf) {
    const int t = threadIdx.x;
    buf[t] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t u = t >= off ? buf[t - off] : 0;
        __syncthreads();
        buf[t] += u;
        __syncthreads();
    }
    const int64_t r = buf[t] - v;
    __syncthreads();
    return r;
}

// One workgroup: per chunk, the rank of its first tied entry (eq_base) and the
// output offset of its first selected entry (out_base).  A chunk takes all its
// entries above T and its tied entries whose global tie rank is below the
// number of ties still to take.
__global__ void __launch_bounds__(1024) k_sel_scan(const int2 *__restrict__ cnt, int64_t nblk,
                                                   const SelState *__restrict__ st, int64_t *__restrict__ eq_base,
                                                   int64_t *__restrict__ out_base) {
    __shared__ int64_t buf[1024];
    const int64_t need = st->remaining;
    const int64_t per = (nblk + 1023) / 1024;
    const int64_t b0 = imin((int64_t)threadIdx.x * per, nblk), b1 = imin(b0 + per, nblk);
    int64_t s = 0;
    for (int64_t b = b0; b < b1; b++) s += cnt[b].y;
    int64_t e = block_exclusive_scan(s, buf);
    int64_t sel = 0;
    for (int64_t b = b0; b < b1; b++) {
        eq_base[b] = e;
        const int64_t take = imin(imax(need - e, 0), cnt[b].y);
        sel += cnt[b].x + take;
        e += cnt[b].y;
    }
    int64_t o = block_exclusive_scan(sel, buf);
    for (int64_t b = b0; b < b1; b++) {
        out_base[b] = o;
        const int64_t take = imin(imax(need - eq_base[b], 0), cnt[b].y);
        o += cnt[b].x + take;
    }
}

struct OpenMap {
    uint64_t fixed; // fixed bits with the open qubits cleared
    int32_t n;
    int32_t q[30];
};

__device__ __forceinline__ int wave_rank(bool f, int &total) {
    const uint64_t m = __ballot(f);
    total = __popcll(m);
    const int lane = threadIdx.x & 63;
    return __popcll(m & ((1ull << lane) - 1ull));
}

// Ordered write: chunk entries in index order, rounds of 256 consecutive ones.
__global__ void __launch_bounds__(256) k_sel_write(const float2 *__restrict__ amps, int64_t n,
                                                   const SelState *__restrict__ st,
                                                   const int64_t *__restrict__ eq_base,
                                                   const int64_t *__restrict__ out_base, OpenMap om, int64_t count,
                                                   uint64_t *__restrict__ out) {
    __shared__ int wtot[2][4];
    const uint64_t T = st->prefix;
    const int64_t need = st->remaining;
    const int64_t base = (int64_t)blockIdx.x * kChunk;
    const int w = threadIdx.x >> 6;
    int64_t eq_run = eq_base[blockIdx.x], sel_run = out_base[blockIdx.x];
    for (int j = 0; j < kChunk / 256; j++) {
        const int64_t i = base + j * 256 + threadIdx.x;
        uint64_t k = 0;
        if (i < n) k = key_of(amps[i]);
        const bool is_eq = i < n && k == T, is_gt = i < n && k > T;
        int te;
        const int re = wave_rank(is_eq, te);
        if ((threadIdx.x & 63) == 0) wtot[0][w] = te;
        __syncthreads();
        int eq_before = re;
        for (int u = 0; u < w; u++) eq_before += wtot[0][u];
        const int eq_round = wtot[0][0] + wtot[0][1] + wtot[0][2] + wtot[0][3];
        const bool sel = is_gt || (is_eq && eq_run + eq_before < need);
        int ts;
        const int rs = wave_rank(sel, ts);
        if ((threadIdx.x & 63) == 0) wtot[1][w] = ts;
        __syncthreads();
        int sel_before = rs;
        for (int u = 0; u < w; u++) sel_before += wtot[1][u];
        const int sel_round = wtot[1][0] + wtot[1][1] + wtot[1][2] + wtot[1][3];
        const int64_t pos = sel_run + sel_before;
        if (sel && pos < count) {
            uint64_t bits = om.fixed;
            for (int b = 0; b < om.n; b++) bits |= (uint64_t)((i >> b) & 1) << om.q[b];
            out[pos] = bits;
        }
        eq_run += eq_round;
        sel_run += sel_round;
        __syncthreads();
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

} // namespace

size_t select_scratch_bytes(int64_t n) {
    const int64_t nblk = (n + kChunk - 1) / kChunk;
    return align256(sizeof(SelState)) + align256(kBins * sizeof(unsigned)) + align256((size_t)nblk * sizeof(int2)) +
           2 * align256((size_t)nblk * sizeof(int64_t));
}

void launch_select_top(const float2 *amps, int n_open, const int32_t *open_q, uint64_t fixed, int64_t count,
                       uint64_t *out, void *work, hipStream_t s) {
    const int64_t n = (int64_t)1 << n_open;
    const int64_t nblk = (n + kChunk - 1) / kChunk;
    char *w = (char *)work;
    SelState *st = (SelState *)w;
    w += align256(sizeof(SelState));
    unsigned *hist = (unsigned *)w;
    w += align256(kBins * sizeof(unsigned));
    int2 *cnt = (int2 *)w;
    w += align256((size_t)nblk * sizeof(int2));
    int64_t *eq_base = (int64_t *)w;
    w += align256((size_t)nblk * sizeof(int64_t));
    int64_t *out_base = (int64_t *)w;
    OpenMap om{};
    om.n = n_open;
    uint64_t open_mask = 0;
    for (int b = 0; b < n_open; b++) {
        om.q[b] = open_q[b];
        open_mask |= 1ull << open_q[b];
    }
    om.fixed = fixed & ~open_mask;
    const unsigned hblocks = (unsigned)std::min<int64_t>((n + 255) / 256, 2048);
    hipLaunchKernelGGL(k_sel_init, dim3(1), dim3(256), 0, s, st, hist, count);
    for (int d = 0; d < kPasses; d++) {
        hipLaunchKernelGGL(k_sel_hist, dim3(hblocks), dim3(256), 0, s, amps, n, kLo[d], kWidth[d], st, hist);
        hipLaunchKernelGGL(k_sel_pick, dim3(1), dim3(256), 0, s, hist, kWidth[d], st);
    }
    hipLaunchKernelGGL(k_sel_count, dim3((unsigned)nblk), dim3(256), 0, s, amps, n, st, cnt);
    hipLaunchKernelGGL(k_sel_scan, dim3(1), dim3(1024), 0, s, cnt, nblk, st, eq_base, out_base);
    hipLaunchKernelGGL(k_sel_write, dim3((unsigned)nblk), dim3(256), 0, s, amps, n, st, eq_base, out_base, om, count,
                       out);
}

} // namespace rqc
