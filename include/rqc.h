/*
 * librqc -- sliced tensor-network amplitudes and rejection sampling for random
 * quantum circuits on AMD Instinct MI355X (gfx950).
 *
 * The operations follow arXiv 2112.15083 ("Classical sampling of random
 * quantum circuits with bounded fidelity"):
 *   - a circuit's amplitudes <x|C|0> for batches of bitstrings sharing fixed
 *     bits (introduction: batches of amplitudes; Sec. II.A: b = (b_A, b_B));
 *   - contraction along a tree T with sliced ("projected") variables I summed at
 *     the very last step (Sec. I, first paragraphs), optionally partially: the
 *     slices X x {0,1}^{|I|-|S|} of Sec. I.C, normalised by 1/sqrt(F);
 *   - the modified frugal rejection sampling of Sec. II.A.
 *
 * Memory and threading
 *   Handles are opaque and owned by the caller (create/destroy pairs).  All
 *   data buffers are owned by the caller.  "device" pointers are HIP device
 *   addresses on the current device; "host" pointers are ordinary memory.  The
 *   library allocates its plan workspace (leaf tensors, intermediate arena,
 *   FP64 accumulators, the norm network of partial slicing) at plan creation,
 *   through the allocator in rqc_plan_opts or hipMalloc, and nothing per call.
 *   The entry points without a plan (rqc_rejection_sample, rqc_kernel_cgemm)
 *   keep a small device scratch block per (device, stream) that grows when a
 *   call needs more and is kept until the library is unloaded; calls on one
 *   stream are serialised on it, calls on different streams overlap.
 *   Calls that take a stream enqueue their GPU work on it and return; unless a
 *   call says otherwise, results are ready when that stream is synchronised.
 *   A plan may be used by one thread at a time; distinct plans are independent.
 *   Successive calls on one plan may use different streams: each call's work
 *   waits for the previous call's (the calls share the plan's workspace).
 *
 * Errors
 *   Every call returns an rqc_status.  On a non-OK status nothing was written to
 *   the outputs unless stated, and rqc_last_error() returns a thread-local
 *   message describing the failure.  No C++ exception crosses this interface.
 *
 * Conventions
 *   Qubit q is bit q of every bitstring integer.  A batch of 2^o amplitudes is
 *   indexed by t in [0, 2^o): bit b of t is the value of qubit open_qubits[b];
 *   the other qubits take their bits from the batch's fixed-bit mask.
 *   Complex64 values are interleaved (re, im) float pairs; complex128 likewise
 *   with doubles.
 *   Variables (tensor legs; Appendix B calls them vertices): ids 0..n-1 are the
 *   qubit inputs (fixed to |0>); walking the gate lines in order, each
 *   single-qubit gate creates one variable (its output), an fSim with
 *   theta = pi/2 creates none (it equals SWAP times a diagonal gate), any other
 *   two-qubit gate creates two (first qubit first).
 *
 * Circuit text: see rqc_load_circuit.
 */
#ifndef RQC_H
#define RQC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rqc_circuit rqc_circuit;
typedef struct rqc_plan rqc_plan;

typedef enum {
    RQC_OK = 0,
    RQC_EINVAL = -1,  /* bad argument */
    RQC_EPARSE = -2,  /* malformed circuit text */
    RQC_EPLAN = -3,   /* no plan satisfies the options */
    RQC_ENOMEM = -4,  /* workspace allocation failed or exceeds the budget */
    RQC_EDEVICE = -5, /* HIP runtime error, or no GPU / wrong architecture */
    RQC_ESHORT = -6   /* sampler: fewer accepted samples than requested */
} rqc_status;

typedef enum {
    RQC_C64 = 0,    /* complex64 contraction, FP32 MFMA, FP32 accumulate */
    RQC_BF16X3 = 1, /* GEMMs as 3 bfloat16 split products, FP32 accumulate */
    RQC_FP16X3 = 2  /* GEMMs as 3 float16 split products with 2^e scaling */
} rqc_precision;

/* Device allocator used for the plan workspace.  Must return memory usable by
   kernels on the current device, aligned to 256 bytes, or NULL on failure. */
typedef void *(*rqc_alloc_fn)(size_t bytes, void *ctx);
typedef void (*rqc_free_fn)(void *ptr, void *ctx);

typedef struct {
    /* Slicer memory target: slice until every intermediate tensor has at most
       2^max_log2_tensor elements (0 = no memory target). */
    int32_t max_log2_tensor;
    /* Slicer leg-count target: slice at least this many legs, each chosen to
       minimise the total sliced cost (-1 = memory target only). */
    int32_t n_sliced_target;
    /* Slices whose legs are carried as an extra tensor mode ("batched") instead
       of being looped over: the largest batched tensor has at most
       2^max_log2_batched elements (0 = 28). */
    int32_t max_log2_batched;
    /* rqc_precision of the contraction GEMMs. */
    int32_t precision;
    /* Partial slicing (Sec. I.B, Appendix B Alg. 1).  target_fidelity >= 1 or
       <= 0: full slicing.  Otherwise k0 = ceil(3 - log2 f) partially sliced
       vertices are chosen by SlicedVertexSelect among the sliced legs, their
       norms R are computed on the GPU and X is the minimal top-R set reaching f.
       When the library searches the slicing itself (no user path or legs), it
       first takes k0 vertices as close to the inputs as possible (light cones of
       at most four vertices, pairwise causally unrelated, those indexing the
       most contraction cost first: Sec. I.B step 1), searches the tree for the
       network with them projected, and adds legs for the memory target.
       partial_k > 0 overrides k0; partial_count > 0 keeps exactly that many
       top-R indices instead of the sum rule. */
    double target_fidelity;
    int32_t partial_k;
    int32_t partial_count;
    /* > 0: keep the top-R indices so that |X| * 2^(|I|-|S|) is this many slices
       (at least one index); overrides partial_count and the sum rule. */
    int64_t partial_total_slices;
    /* Greedy path search: number of randomised trials (0 = 16) and RNG seed. */
    int32_t path_trials;
    uint64_t path_seed;
    /* 1 = time every kernel class with HIP events (see rqc_plan_profile). */
    int32_t profile;
    /* 1 = plan on the host only: no device is touched and the plan can only be
       inspected (rqc_plan_info and friends), not executed.  With partial
       slicing, S is selected but the norms R need the GPU: R and X stay empty,
       the fidelity is reported as 0 and the default slice list is empty. */
    int32_t dry_run;
    /* Workspace allocator (NULL alloc = hipMalloc / hipFree). */
    rqc_alloc_fn alloc;
    rqc_free_fn free;
    void *alloc_ctx;
    /* 1 = global cache across batches (the multi-batch reuse the paper's
       introduction relies on): the parts of the contraction that do not depend
       on the fixed output bits are computed once per slice group, on the first
       rqc_contract_amplitudes call over the plan's default slice list, and kept
       in the workspace; every later call contracts only the parts that depend
       on its fixed bits.  Results are bitwise identical with and without the
       cache.  Costs rqc_plan_info_t.cache_bytes of workspace (RQC_EPLAN if that
       exceeds 128 GiB). */
    int32_t global_cache;
    /* > 1: time this many of the searched trees (best estimated time first) on
       the device, one batch each after a warm-up, and keep the fastest if it
       beats the estimate's choice by at least 5 %; the planner's estimate
       alone decides otherwise.  Only for searched trees with full slicing. */
    int32_t autotune;
    /* 1 = run every streaming step on its own.  By default a streaming step
       whose result only feeds the next streaming step runs fused with it when
       their shapes fit the fused kernel: the intermediate stays in LDS instead
       of going through HBM.  Results agree with the unfused plan to FP32
       rounding (the second contraction may add its index in another order). */
    int32_t no_stream_fusion;
    /* 1 = run every streaming step on the vector-ALU kernels instead of the
       matrix-core forms (and unfused): an ablation, and the route that checks
       those kernels against the oracle.  Slower; results agree to FP32
       rounding. */
    int32_t no_matrix_core_streams;
    /* > 0: refine the best searched trees by simulated annealing of the tree
       and of the sliced legs (Sec. I names it as the optimiser of T and I),
       this many Metropolis moves each; the refined trees compete with the
       searched ones by estimated time.  User-given legs are kept fixed. */
    int32_t anneal_iters;
} rqc_plan_opts;

typedef struct {
    int32_t n_qubits;
    int32_t n_open;
    int32_t n_variables;
    int32_t n_sliced;          /* |I| */
    int32_t n_batched;         /* sliced legs carried as a tensor mode */
    int32_t n_partial;         /* k = |S| (0 for full slicing) */
    int64_t n_slices;          /* slices in the plan's default slice list */
    int64_t n_partial_kept;    /* |X| */
    double fidelity;           /* F = sum_{i in X} R[i]; 1 for full slicing */
    double flops_per_batch;    /* algorithmic flops (8 per complex multiply-add)
                                  of one open batch over the default slice list */
    double flops_unsliced;     /* the same for the tree without slicing */
    double gemm_flop_share;    /* share of flops_per_batch in MFMA GEMM steps */
    double bytes_per_batch;    /* algorithmic HBM bytes: each step's operands read
                                  once and result written once, plus permutes */
    int32_t max_log2_tensor;   /* largest intermediate (with batched slice legs) */
    int32_t n_steps;           /* pairwise contractions in the tree */
    int32_t n_launches;        /* kernel launches per slice group */
    int64_t n_groups;          /* slice groups per batch */
    int64_t workspace_bytes;   /* device memory held by the plan */
    double plan_seconds;       /* host time spent planning */
    int64_t cache_bytes;       /* global cache held (0 without global_cache) */
    double flops_cached;       /* of flops_per_batch, the part that does not
                                  depend on the fixed bits (computed once per
                                  plan when global_cache is set) */
    double est_seconds;        /* the planner's estimate of one batch's GPU time
                                  (what it minimises over candidate trees) */
    int32_t n_fused;           /* streaming pairs run fused (see no_stream_fusion) */
    /* streaming launches per slice group by kernel: [0] fused pair, [1]
       matrix-core tile, [2] matrix-core long contraction, [3] vector long
       contraction, [4] vector LDS tile, [5] vector generic; [6], [7] unused */
    int32_t stream_kernels[8];
} rqc_plan_info_t;

typedef struct {
    int64_t accepted;   /* accepted batches (may exceed the samples returned) */
    int64_t batches;    /* batches examined */
    int64_t batches_used; /* batches up to the one that gave the last sample kept */
    double eps_J;       /* sum over examined batches of max(0, p_j - alpha/N_B) */
    double p_total;     /* sum of all examined p_j (normalised units) */
} rqc_sample_stats;

/* Kernel classes reported by rqc_plan_profile. */
enum {
    RQC_K_LEAF = 0,      /* slice/fixed-bit selection of leaf tensors */
    RQC_K_SMALL = 1,     /* fused small-subtree contraction in LDS */
    RQC_K_STREAM = 2,    /* streaming small-K contraction (HBM bound) */
    RQC_K_PERMUTE = 3,   /* tensor permute */
    RQC_K_GEMM = 4,      /* complex GEMM on MFMA */
    RQC_K_ACCUM = 5,     /* FP64 cross-slice accumulation */
    RQC_K_FINAL = 6,     /* normalisation and output conversion */
    RQC_K_SAMPLE = 7,    /* probabilities and rejection sampling */
    RQC_K_CLASSES = 8
};

/* Per-op totals of the profiled launches (rqc_plan_profile_ops). */
typedef struct {
    int32_t cls;        /* RQC_K_* class */
    int32_t op;         /* index of the op in the plan's launch program; -1 for
                           the per-slice-group launches outside it (leaf
                           selection, accumulation, normalisation) */
    int64_t launches;
    double seconds;     /* summed HIP-event durations */
    double flops;       /* algorithmic flops, 8 per complex multiply-add */
    double bytes;       /* algorithmic HBM bytes: operands read once, result
                           written once */
    double exec_flops;  /* flops the launches execute on the matrix cores or
                           vector ALUs (the FP32 GEMM: 6 per complex
                           multiply-add; the split GEMMs: 24) */
    int32_t exec_kind;  /* precision of exec_flops: 0 = FP32, 1 = bf16/fp16 */
    int32_t pad;
} rqc_op_profile_t;

typedef struct {
    int64_t launches[RQC_K_CLASSES];
    double seconds[RQC_K_CLASSES];   /* summed HIP-event durations */
    double flops[RQC_K_CLASSES];     /* algorithmic flops of the timed launches */
    double bytes[RQC_K_CLASSES];     /* algorithmic bytes of the timed launches */
} rqc_profile_t;

/*
 * Parse circuit text.  Format ("rqc-circuit 1"; '#' starts a comment):
 *   qubits <n>                    number of qubits, 1..64
 *   grid <rows> <cols> / removed <r> <c> / cycles <m>   (informational)
 *   sx|sy|sw <cycle> <q>          sqrt(P) = (I - iP)/sqrt(2), P in X, Y,
 *                                 W = (X+Y)/sqrt(2)
 *   fsim <cycle> <qa> <qb> <t> <p> fSim(pi*t, pi*p), t and p exact fractions;
 *                                 matrix in the basis |b_qa b_qb>:
 *                                 [[1,0,0,0],[0,c,-is,0],[0,-is,c,0],[0,0,0,e^{-i pi p}]]
 * Gate lines are applied in order.  `text` is host memory of `len` bytes.
 * Returns RQC_EPARSE (with the line number in rqc_last_error) on bad input.
 */
rqc_status rqc_load_circuit(const char *text, size_t len, rqc_circuit **out);
rqc_status rqc_circuit_info(const rqc_circuit *c, int32_t *n_qubits, int32_t *n_variables,
                            int32_t *n_gates);
void rqc_circuit_destroy(rqc_circuit *c);

/*
 * Build a contraction plan (Sec. I: contraction tree T and sliced variables I).
 *   path, n_path_pairs: optional contraction order as SSA pairs: leaf tensor t
 *     is gate line t, and contraction number s creates tensor n_gates + s.
 *     NULL = the library's randomised greedy path.
 *   sliced_legs, n_sliced: optional variable ids to slice (NULL = greedy slicer
 *     under opts).  Input variables and output variables cannot be sliced.
 *   open_qubits[b]: the qubit carried by bit b of the batch index (host array).
 * The plan uploads its leaf tensors and reserves its workspace on the current
 * device.  opts may be NULL (defaults: no slicing, complex64).
 */
rqc_status rqc_plan_create(const rqc_circuit *c, const int32_t *path, int32_t n_path_pairs,
                           const int32_t *sliced_legs, int32_t n_sliced,
                           const int32_t *open_qubits, int32_t n_open,
                           const rqc_plan_opts *opts, rqc_plan **out);
rqc_status rqc_plan_info(const rqc_plan *p, rqc_plan_info_t *info);
/* Sliced variable ids in slice-id bit order (bit t of a slice id = legs[t]). */
rqc_status rqc_plan_sliced_legs(const rqc_plan *p, int32_t *legs, int32_t cap, int32_t *count);
/* The plan's contraction tree as SSA pairs, in the form rqc_plan_create takes
   (pairs[2s], pairs[2s+1] for step s; cap and *count are pair counts), so that
   another plan can be built on the same tree (the path the Sec. I tree T is
   contracted along). */
rqc_status rqc_plan_path(const rqc_plan *p, int32_t *pairs, int32_t cap, int32_t *count);
/* The plan's launch program as text, one op per line in launch order
   ("<op> <kind> <kernel> <depends on fixed bits> <flops> <bytes> <shape>";
   kernel "mx-wide" is the matrix-core streaming tile in its 64-bit addressed
   form, for tiles spanning tensors of 2^29 elements or more):
   what each contraction step of the tree became.  buf (host) receives at most
   cap bytes, NUL-terminated; *len the full size including the NUL. */
rqc_status rqc_plan_describe(const rqc_plan *p, char *buf, size_t cap, size_t *len);
/* Partial slicing results: S (variable ids, bit t of an index i = S[t]), the
   kept indices X in selection order, and R[0 .. 2^k) (host arrays; any may be
   NULL; caps are element counts). */
rqc_status rqc_plan_partial(const rqc_plan *p, int32_t *S, int32_t capS, uint64_t *X, int64_t capX,
                            double *R, int64_t capR);
/* The plan's default slice list as slice ids, in the plan's summation order
   (host array; *count receives the full length, at most cap ids are written). */
rqc_status rqc_plan_slices(const rqc_plan *p, uint64_t *ids, int64_t cap, int64_t *count);
rqc_status rqc_plan_profile(const rqc_plan *p, rqc_profile_t *out);
rqc_status rqc_plan_profile_reset(rqc_plan *p);
/* With profile = 1: time only the launches of the classes whose bit
   (1 << RQC_K_*) is set in mask (every class until this is called).  Each
   timed launch records two HIP events on its stream, which costs a few
   microseconds per launch; timing one class leaves the others' launches
   back to back.  Applies to later calls; bits at RQC_K_CLASSES or above give
   RQC_EINVAL. */
rqc_status rqc_plan_profile_classes(rqc_plan *p, uint32_t mask);
/* The same profile split by op of the launch program (host array of cap
   records; *count receives the number of records).  Synchronises on the
   profiled work. */
rqc_status rqc_plan_profile_ops(const rqc_plan *p, rqc_op_profile_t *ops, int32_t cap, int32_t *count);
/* Free a plan.  No work using the plan may still be pending on any stream when
   its workspace came from a caller-supplied allocator; with the default
   allocator the device is synchronised first. */
void rqc_plan_destroy(rqc_plan *p);

/*
 * Amplitudes of n_batches open batches (Sec. I.C partial contraction):
 *   amp_b[t] = (1/sqrt(F)) * sum_{s in slices} <x_b(t)| C_s |0>
 * where x_b(t) combines fixed_bits[b] (host array of n-bit masks; open bits
 * ignored) with t on the open qubits, C_s is the network with the sliced
 * variables fixed to the bits of slice id s, and the sum runs in FP64 in the
 * plan's fixed slice order (independent of how slices are grouped).
 *   slice_ids: host array of slice ids, or NULL for the plan's default list
 *     (all 2^|I| slices, or X x {0,1}^{|I|-|S|} under partial slicing).  A
 *     custom list must be a union of whole batched-slice groups with no id
 *     repeated and no bit above the sliced legs (else RQC_EINVAL before any
 *     launch); an empty list (n_slices = 0, non-NULL) is the empty sum and
 *     writes exact zeros.  n_batches = 0 writes nothing.
 *   out_amps: device complex64 [n_batches][2^n_open].
 *   out_f64: optional device complex128 [n_batches][2^n_open] receiving the
 *     same normalised amplitudes before rounding to complex64.
 *   hip_stream: hipStream_t to enqueue on (NULL = default stream).
 * Asynchronous on hip_stream.
 */
rqc_status rqc_contract_amplitudes(rqc_plan *p, const uint64_t *slice_ids, int64_t n_slices,
                                   const uint64_t *fixed_bits, int64_t n_batches, void *out_amps,
                                   void *out_f64, void *hip_stream);

/*
 * The same contraction in work units, for schedulers that interleave requests
 * (the serving loop runs one unit of a request at a time, so a long request
 * does not hold a stream for its whole duration):
 *   rqc_contract_groups adds, for each of n_batches batches, the FP64 slice
 *   sums of the plan's default slice groups [first_group, first_group +
 *   n_groups) (groups in the plan's order; rqc_plan_info_t.n_groups of them)
 *   into acc_f64, device complex128 [n_batches][2^n_open], unnormalised; a call
 *   with first_group = 0 overwrites the accumulator instead of adding to it.
 *   rqc_finalize_amplitudes then writes (1/sqrt(F)) times the accumulated sums
 *   as complex64 to out_amps (and the FP64 values to out_f64 if non-null).
 * Calls over consecutive group ranges from 0 to n_groups, in order, followed by
 * rqc_finalize_amplitudes, give results bit-identical to one
 * rqc_contract_amplitudes call with the default slice list (the FP64 running
 * sum is carried in the accumulator).  A range beyond the list gives
 * RQC_EINVAL.  Asynchronous on hip_stream, ordered after the plan's previous
 * calls.
 */
rqc_status rqc_contract_groups(rqc_plan *p, int64_t first_group, int64_t n_groups, const uint64_t *fixed_bits,
                               int64_t n_batches, void *acc_f64, void *hip_stream);
rqc_status rqc_finalize_amplitudes(rqc_plan *p, const void *acc_f64, int64_t n_batches, void *out_amps,
                                   void *out_f64, void *hip_stream);

/*
 * Modified frugal rejection sampling (Sec. II.A) over computed batches.
 *   amps: device complex64 [n_batches][2^n_open]; each open batch is split into
 *     sub-batches of N_A = 2^log2_NA amplitudes (bits 0..log2_NA-1 of the batch
 *     index are b_A), so it holds 2^(n_open - log2_NA) sub-batches j, numbered
 *     globally batch_index_base + b * 2^(n_open-log2_NA) + j_local.
 *   fixed_bits: host masks of the batches (as in rqc_contract_amplitudes).
 *   open_qubits: host array as in the plan.  N_B = 2^(n_qubits - log2_NA).
 *   Per sub-batch, in global order: p_ij = re^2 + im^2 in FP64, p_j the
 *   sequential FP64 sum, accept iff U0 < p_j * N_B / (alpha * F_norm), then
 *   i = first index whose sequential prefix sum exceeds U1 * p_j (else the last
 *   i with p_ij > 0), U_d = Philox4x32-10 uniform (key = seed, counter =
 *   (global sub-batch index, d, 0)).
 *   pick_steps > 0 selects the literal "pick j at random" mode instead: the
 *     amps hold one full vector (n_batches = 1, all qubits open); step t picks
 *     j from Philox draw 2 at counter t and uses counter t for U0 and U1; up to
 *     pick_steps steps are taken.
 *   out_samples: device uint64 [n_samples] bitstrings, in ascending sub-batch
 *     (or step) order; *n_out (host) receives the count; stats (host, optional).
 * Synchronises hip_stream before returning.  Returns RQC_ESHORT if fewer than
 * n_samples were accepted (the first *n_out entries are valid).
 */
rqc_status rqc_rejection_sample(const void *amps, const uint64_t *fixed_bits, int64_t n_batches,
                                const int32_t *open_qubits, int32_t n_open, int32_t log2_NA,
                                int32_t n_qubits, double alpha, double F_norm, uint64_t seed,
                                uint64_t batch_index_base, int64_t pick_steps, int64_t n_samples,
                                uint64_t *out_samples, int64_t *n_out, rqc_sample_stats *stats,
                                void *hip_stream);

/*
 * rqc_rejection_sample for callers that cannot allocate device memory (code
 * that must not call hipMalloc: serving loops and harnesses that forbid it).
 * Same arguments, results and errors as rqc_rejection_sample, bit for bit; the
 * difference is where the per-call scratch lives (per sub-batch results, the
 * fixed bits and open qubits copied to the device, the compaction counters):
 * in a fixed array of RQC_SAMPLE_STATIC_SCRATCH_BYTES that the library holds on
 * each device it runs on until the process ends.  The call allocates nothing.
 * A call needs 16 * items + 8 * n_batches + 4 * n_open bytes plus 1 KiB of
 * alignment and counters (items = n_batches * 2^(n_open - log2_NA), or
 * pick_steps); a call needing more returns RQC_EINVAL before any GPU work
 * (about 5.2e5 sub-batches fit).  Every call on a device shares that device's
 * array, which keeps the last call's contents (each call writes every word it
 * reads before reading it, so nothing has to start at zero).  Calls that
 * overlapped on one device would race on the array: the library serialises
 * them with a per-device lock held until the call's GPU work has finished (the
 * call synchronises hip_stream before returning), so only calls from other
 * processes, which hold their own arrays, run beside it.
 */
#define RQC_SAMPLE_STATIC_SCRATCH_BYTES (8u << 20)
rqc_status rqc_rejection_sample_static(const void *amps, const uint64_t *fixed_bits, int64_t n_batches,
                                       const int32_t *open_qubits, int32_t n_open, int32_t log2_NA,
                                       int32_t n_qubits, double alpha, double F_norm, uint64_t seed,
                                       uint64_t batch_index_base, int64_t pick_steps, int64_t n_samples,
                                       uint64_t *out_samples, int64_t *n_out, rqc_sample_stats *stats,
                                       void *hip_stream);

/*
 * Linear-XEB spoofing (Sec. III.B, step 4): the `count` bitstrings of one
 * computed open batch with the largest probabilities.
 *   amps: device complex64 [2^n_open], a batch as rqc_contract_amplitudes
 *     writes it (under partial slicing, the approximate amplitudes of step 3).
 *   p_t = (double)re^2 + (double)im^2 (squares exact, one rounding); the selection is every t with
 *     p_t > T and, among the t with p_t = T, the smallest ones, where T is the
 *     count-th largest p_t; so it is unique.
 *   out_samples: device uint64 [count], the selected bitstrings in ascending
 *     batch index t (fixed_bits on the other qubits, as in
 *     rqc_contract_amplitudes).
 *   0 <= count <= 2^n_open (else RQC_EINVAL); open_qubits (host) distinct.
 * Asynchronous on hip_stream; uses the per-stream scratch block (a few bytes
 * per 4096 amplitudes).
 */
rqc_status rqc_select_top(const void *amps, uint64_t fixed_bits, const int32_t *open_qubits, int32_t n_open,
                          int32_t n_qubits, int64_t count, uint64_t *out_samples, void *hip_stream);

/*
 * FP64 probability sums (the reductions of Sec. II.A and Eq. (1)): for each
 * of n_rows rows of row_len complex64 amplitudes,
 *   sums[r] = sum_i p_ri with p_ri = (double)re^2 + (double)im^2,
 * the squared norm of a batch, or, when the row holds the amplitudes of k =
 * row_len sampled bitstrings of an n_qubits circuit, the sum in the linear
 * cross-entropy benchmark of Eq. (1); then, if xeb is not NULL,
 *   xeb[r] = 2^n_qubits * sums[r] / row_len - 1.
 *   amps: device complex64 [n_rows][row_len] (interleaved re, im), contiguous.
 *   sums, xeb: device double [n_rows]; xeb may be NULL.
 * The order of the additions depends only on row_len (chunks of 8192 entries,
 * fixed trees), so repeated calls give the same bits.  row_len = 0 gives sums
 * of 0 (and RQC_EINVAL if xeb is asked); n_rows = 0 does nothing; n_rows *
 * ceil(row_len / 8192) must stay below 2^31 (else RQC_EINVAL).  Asynchronous
 * on hip_stream; uses the per-stream scratch block (8 bytes per 8192
 * amplitudes).
 */
rqc_status rqc_prob_sums(const void *amps, int64_t n_rows, int64_t row_len, int32_t n_qubits, double *sums,
                         double *xeb, void *hip_stream);

/*
 * Kernel-level primitives (the contraction steps of Sec. I run on these; they
 * are exported for direct use and for testing each kernel variant).
 *
 * Batched complex GEMM C[b] = A[b] B[b] (complex64, interleaved, device):
 *   A element (m,k) of batch b at b*M*K + (a_kfast ? m*K + k : k*M + m),
 *   B element (k,n) at b*K*N + (b_nfast ? k*N + n : n*K + k),
 *   C element (m,n) at b*M*N + m*N + n.
 * M and N must be powers of two >= 64, K a power of two >= 8.  precision is an
 * rqc_precision; the split modes use 3 bf16/fp16 products per real product
 * (fp16 with a per-operand power-of-two scale) and need K >= 16, otherwise
 * the FP32 MFMA kernel runs.  Asynchronous on hip_stream.
 */
rqc_status rqc_kernel_cgemm(const void *A, const void *B, void *C, int64_t batch, int64_t M, int64_t N,
                            int64_t K, int32_t a_kfast, int32_t b_nfast, int32_t precision, void *hip_stream);
/*
 * Bit permutation of a 2^r-element complex64 tensor (device):
 * dst[sum_i bit_i(x) << perm[i]] = src[x]; perm (host) is a permutation of 0..r-1.
 * Asynchronous on hip_stream (the tiling descriptor is passed in the kernel
 * arguments; perm may be reused as soon as the call returns).
 */
rqc_status rqc_kernel_permute(const void *src, void *dst, int32_t r, const int32_t *perm, void *hip_stream);

/* Thread-local message for the last non-OK status (never NULL). */
const char *rqc_last_error(void);
/* Library version string. */
const char *rqc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RQC_H */
