// Modified frugal rejection sampling (Sec. II.A) on the GPU.
//
// Per batch j of N_A amplitudes: p_ij = re^2 + im^2 in FP64 (products of FP32
// values are exact in FP64), p_j = sequential FP64 sum, accept iff
// U0 < p_j * N_B / (alpha * F_norm) (this is t_j = min(1, p_j N_B / alpha) of
// step 2, with the amplitudes' squared norm F_norm divided out), then draw i as
// the first index whose sequential prefix sum exceeds U1 * p_j (step 3).
// U_d comes from Philox4x32-10 (Salmon et al., SC'11): key = seed, counter =
// (stream index low, high, d, 0), U = (w1:w0 >> 11) * 2^-53.
// Accepted samples are compacted in ascending batch (or step) order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "kernels.hpp"

namespace rqc {

struct SubResult {
    double pj;
    int32_t accept;
    int32_t idx;
};

__device__ __forceinline__ void philox_round(uint32_t c[4], uint32_t k0, uint32_t k1) {
    const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
    const uint32_t hi0 = __umulhi(m0, c[0]), lo0 = m0 * c[0];
    const uint32_t hi1 = __umulhi(m1, c[2]), lo1 = m1 * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n1 = lo1, n2 = hi0 ^ c[3] ^ k1, n3 = lo0;
    c[0] = n0;
    c[1] = n1;
    c[2] = n2;
    c[3] = n3;
}

__device__ __forceinline__ uint64_t philox_raw64(uint64_t seed, uint64_t stream, uint32_t draw) {
    uint32_t c[4] = {(uint32_t)stream, (uint32_t)(stream >> 32), draw, 0u};
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        philox_round(c, k0, k1);
    }
    return ((uint64_t)c[1] << 32) | (uint64_t)c[0];
}

__device__ __forceinline__ double philox_u53(uint64_t seed, uint64_t stream, uint32_t draw) {
    return (double)(philox_raw64(seed, stream, draw) >> 11) * 0x1.0p-53;
}

__device__ __forceinline__ double prob(float2 a) {
    const double re = (double)a.x, im = (double)a.y;
    return re * re + im * im;
}

// One thread per batch (batches mode) or per step (pick mode).
__global__ void __launch_bounds__(256) k_sample_batches(const float2 *__restrict__ amps, int64_t n_items, int log2_na,
                                                        int log2_nb, double c, uint64_t seed, uint64_t base,
                                                        int pick, SubResult *__restrict__ res) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_items) return;
    const int na = 1 << log2_na;
    int64_t j;
    uint64_t stream;
    if (pick) {
        const uint64_t r = philox_raw64(seed, (uint64_t)t, 2u);
        j = log2_nb > 0 ? (int64_t)(r >> (64 - log2_nb)) : 0;
        stream = (uint64_t)t;
    } else {
        j = t;
        stream = base + (uint64_t)t;
    }
    const float2 *a = amps + j * na;
    double pj = 0.0;
    for (int i = 0; i < na; i++) pj = pj + prob(a[i]);
    const double u0 = philox_u53(seed, stream, 0u);
    SubResult r;
    r.pj = pj;
    r.accept = u0 < pj * c ? 1 : 0;
    r.idx = -1;
    if (r.accept) {
        const double target = philox_u53(seed, stream, 1u) * pj;
        double s = 0.0;
        int last = -1;
        for (int i = 0; i < na; i++) {
            const double p = prob(a[i]);
            s = s + p;
            if (p > 0) last = i;
            if (s > target) {
                r.idx = i;
                break;
            }
        }
        if (r.idx < 0) r.idx = last;
        // record the batch for pick mode in the upper bits of the index word
    }
    if (pick) r.idx = r.accept ? (int32_t)((j << log2_na) | r.idx) : -1;
    res[t] = r;
}

struct CompactStats {
    int64_t accepted;
    int64_t used;
    int64_t n_out;
    double eps_J;
    double p_total;
};

// Single workgroup: ordered compaction of accepted items and the statistics.
__global__ void __launch_bounds__(1024) k_compact(const SubResult *__restrict__ res, int64_t n_items, int log2_na,
                                                  int64_t sub_per_batch, const uint64_t *__restrict__ fixed,
                                                  const int32_t *__restrict__ open_q, int n_open, int pick,
                                                  int64_t n_samples, double cap, double f_norm,
                                                  uint64_t *__restrict__ out, CompactStats *__restrict__ st) {
    __shared__ int64_t scan[1024];
    __shared__ int64_t s_base;
    __shared__ int64_t s_used;
    const int tid = threadIdx.x;
    if (tid == 0) {
        s_base = 0;
        s_used = n_items;
    }
    __syncthreads();
    uint64_t open_mask = 0;
    for (int b = 0; b < n_open; b++) open_mask |= 1ull << open_q[b];
    for (int64_t c0 = 0; c0 < n_items; c0 += 1024) {
        const int64_t item = c0 + tid;
        const int f = (item < n_items && res[item].accept) ? 1 : 0;
        scan[tid] = f;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) { // Hillis-Steele inclusive scan
            int64_t v = tid >= off ? scan[tid - off] : 0;
            __syncthreads();
            scan[tid] += v;
            __syncthreads();
        }
        const int64_t pos = s_base + scan[tid] - f;
        if (f && pos < n_samples) {
            int64_t open_index, batch;
            if (pick) {
                open_index = res[item].idx;
                batch = 0;
            } else {
                batch = item / sub_per_batch;
                open_index = ((item % sub_per_batch) << log2_na) | res[item].idx;
            }
            uint64_t bits = fixed[batch] & ~open_mask;
            for (int b = 0; b < n_open; b++)
                if ((open_index >> b) & 1) bits |= 1ull << open_q[b];
            out[pos] = bits;
            if (pos == n_samples - 1) s_used = item + 1;
        }
        __syncthreads();
        if (tid == 1023) s_base += scan[1023];
        __syncthreads();
    }
    if (tid == 0) {
        st->accepted = s_base;
        st->used = s_used;
        st->n_out = s_base < n_samples ? s_base : n_samples;
        double e = 0.0, pt = 0.0;
        const int64_t lim = pick ? s_used : n_items;
        for (int64_t i = 0; i < lim; i++) {
            const double p = res[i].pj / f_norm;
            pt = pt + p;
            const double d = p - cap;
            if (d > 0) e = e + d;
        }
        st->eps_J = e;
        st->p_total = pt;
    }
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Scratch layout of one call: per-item results, the batches' fixed bits, the
// open qubits, the statistics (each 256-byte aligned).
size_t sampler_scratch_bytes(int64_t n_items, int64_t n_batches, int n_open) {
    return align256((size_t)std::max<int64_t>(n_items, 1) * sizeof(SubResult)) +
           align256((size_t)std::max<int64_t>(n_batches, 1) * sizeof(uint64_t)) +
           align256((size_t)std::max(n_open, 1) * sizeof(int32_t)) + align256(sizeof(CompactStats));
}

hipError_t run_sampler(const float2 *amps, const uint64_t *fixed, int64_t n_batches, const int32_t *open_q,
                       int n_open, int log2_na, int n_qubits, double alpha, double f_norm, uint64_t seed,
                       uint64_t base, int64_t pick_steps, int64_t n_samples, uint64_t *out, int64_t *n_out,
                       rqc_sample_stats *stats, void *work, hipStream_t s) {
    const int pick = pick_steps > 0;
    const int64_t sub_per_batch = (int64_t)1 << (n_open - log2_na);
    const int64_t n_items = pick ? pick_steps : n_batches * sub_per_batch;
    const int log2_nb = n_qubits - log2_na;
    char *w = (char *)work;
    SubResult *res = (SubResult *)w;
    w += align256((size_t)std::max<int64_t>(n_items, 1) * sizeof(SubResult));
    uint64_t *d_fixed = (uint64_t *)w;
    w += align256((size_t)std::max<int64_t>(n_batches, 1) * sizeof(uint64_t));
    int32_t *d_open = (int32_t *)w;
    w += align256((size_t)std::max(n_open, 1) * sizeof(int32_t));
    CompactStats *cst = (CompactStats *)w;
    // the host arrays are read by these copies before the stream is synchronised below
    hipError_t e = hipSuccess;
    if (n_batches > 0) e = hipMemcpyAsync(d_fixed, fixed, (size_t)n_batches * sizeof(uint64_t), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && n_open > 0)
        e = hipMemcpyAsync(d_open, open_q, (size_t)n_open * sizeof(int32_t), hipMemcpyHostToDevice, s);
    const double c = std::ldexp(1.0, log2_nb) / (alpha * f_norm);
    const double cap = alpha / std::ldexp(1.0, log2_nb);
    if (e == hipSuccess && n_items > 0) {
        hipLaunchKernelGGL(k_sample_batches, dim3((unsigned)((n_items + 255) / 256)), dim3(256), 0, s, amps,
                           n_items, log2_na, log2_nb, c, seed, base, pick, res);
    }
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_compact, dim3(1), dim3(1024), 0, s, res, n_items, log2_na, sub_per_batch, d_fixed,
                           d_open, n_open, pick, n_samples, cap, f_norm, out, cst);
        e = hipGetLastError();
    }
    CompactStats h{};
    if (e == hipSuccess) e = hipMemcpyAsync(&h, cst, sizeof(h), hipMemcpyDeviceToHost, s);
    // always wait: the copies above read host memory owned by the caller
    const hipError_t es = hipStreamSynchronize(s);
    if (e == hipSuccess) e = es;
    if (e != hipSuccess) return e;
    *n_out = h.n_out;
    if (stats) {
        stats->accepted = h.accepted;
        stats->batches = pick ? h.used : n_items;
        stats->batches_used = h.used;
        stats->eps_J = h.eps_J;
        stats->p_total = h.p_total;
    }
    return hipSuccess;
}

// FP64 probability sums over rows of amplitudes: the squared norm of a batch,
// and the sum in the linear XEB of Eq. (1) when a row holds the amplitudes of
// k sampled bitstrings (XEB = 2^n * sum / k - 1).  The order of the additions
// depends only on row_len, so every run gives the same bits: a row splits into
// chunks of kSumChunk entries; thread t of a chunk adds entries t, t + 256, ...
// in turn, then the 256 thread sums are combined by a fixed halving tree; the
// chunk sums of a row are combined the same way by one workgroup.
constexpr int kSumThreads = 256;
constexpr int64_t kSumChunk = 8192;

__device__ __forceinline__ double block_tree_sum(double v, double *lds) {
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int h = kSumThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) lds[threadIdx.x] = lds[threadIdx.x] + lds[threadIdx.x + h];
        __syncthreads();
    }
    return lds[0];
}

// One workgroup per (row, chunk); block b = row * nchunk + chunk.
__global__ void __launch_bounds__(kSumThreads) k_prob_chunks(const float2 *__restrict__ amps, int64_t row_len,
                                                             int64_t nchunk, double *__restrict__ part) {
    __shared__ double lds[kSumThreads];
    const int64_t b = blockIdx.x;
    const int64_t row = b / nchunk, c = b - row * nchunk;
    const float2 *a = amps + row * row_len;
    const int64_t lo = c * kSumChunk, hi = lo + kSumChunk < row_len ? lo + kSumChunk : row_len;
    double s = 0.0;
#pragma unroll 8
    for (int64_t e = lo + threadIdx.x; e < hi; e += kSumThreads) s = s + prob(a[e]);
    s = block_tree_sum(s, lds);
    if (threadIdx.x == 0) part[b] = s;
}

// One workgroup per row: the row's chunk sums, then its XEB when asked.
__global__ void __launch_bounds__(kSumThreads) k_prob_rows(const double *__restrict__ part, int64_t nchunk,
                                                           int64_t row_len, int n_qubits, double *__restrict__ sums,
                                                           double *__restrict__ xeb) {
    __shared__ double lds[kSumThreads];
    const int64_t row = blockIdx.x;
    double s = 0.0;
    for (int64_t c = threadIdx.x; c < nchunk; c += kSumThreads) s = s + part[row * nchunk + c];
    s = block_tree_sum(s, lds);
    if (threadIdx.x == 0) {
        sums[row] = s;
        if (xeb) xeb[row] = ldexp(s / (double)row_len, n_qubits) - 1.0;
    }
}

size_t prob_sums_scratch_bytes(int64_t n_rows, int64_t row_len) {
    const int64_t nchunk = (row_len + kSumChunk - 1) / kSumChunk;
    return align256((size_t)(n_rows * nchunk) * sizeof(double));
}

void launch_prob_sums(const float2 *amps, int64_t n_rows, int64_t row_len, int n_qubits, double *sums, double *xeb,
                      void *work, hipStream_t s) {
    const int64_t nchunk = (row_len + kSumChunk - 1) / kSumChunk;
    double *part = (double *)work;
    if (nchunk > 0) hipLaunchKernelGGL(k_prob_chunks, dim3((unsigned)(n_rows * nchunk)), dim3(kSumThreads), 0, s,
                                       amps, row_len, nchunk, part);
    hipLaunchKernelGGL(k_prob_rows, dim3((unsigned)n_rows), dim3(kSumThreads), 0, s, (const double *)part, nchunk,
                       row_len, n_qubits, sums, xeb);
}

// ------------------------------------------------------------ fixed scratch
// The scratch of rqc_rejection_sample_static: one array per device, held until
// the process ends.  On the host its name is a stand-in, not a device address,
// so host code never passes it to a kernel or a copy; it takes the address
// hipGetSymbolAddress returns for the current device (each device holds its own
// copy of the array at its own address) and passes that.
static __device__ __align__(256) unsigned char scratch[RQC_SAMPLE_STATIC_SCRATCH_BYTES];

static std::mutex g_static_mu;
static void *g_static_ptr[kMaxDevices] = {};
static std::mutex g_static_call_mu[kMaxDevices];

hipError_t static_scratch(void **ptr, std::mutex **call_mu) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_static_ptr[dev] = p;
    }
    *ptr = g_static_ptr[dev];
    *call_mu = &g_static_call_mu[dev];
    return hipSuccess;
}

} // namespace rqc
