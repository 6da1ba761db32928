// C-ABI of librqc: circuit handles, plan creation and upload, the slice-group
// executor, the sampler entry point and the kernel-level primitives.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>

#include "kernels.hpp"

namespace rqc {

static thread_local std::string g_err = "no error";

void fail(rqc_status code, const std::string &msg) { throw Error{code, msg}; }

#define HIP_OK(x)                                                                                   \
    do {                                                                                            \
        hipError_t e_ = (x);                                                                        \
        if (e_ != hipSuccess) rqc::fail(RQC_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

static void check_device() {
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        fail(RQC_EDEVICE, std::string("librqc is built for gfx950; current device is ") + prop.gcnArchName);
}

// Device scratch for the entry points that have no plan (the sampler and the
// kernel-level primitives): one block per (device, stream), grown
// geometrically with hipMalloc when a call needs more and never freed while
// the library is loaded (retired blocks are kept rather than freed, since
// hipFree waits for the whole device).  A call holds its block's lock until
// its work on the stream no longer reads it, so concurrent calls on one stream
// from several threads are serialised and calls on different streams overlap.
struct StreamScratch {
    std::mutex mu;
    void *ptr = nullptr;
    size_t bytes = 0;
    std::vector<void *> retired;
};

static StreamScratch &stream_scratch(hipStream_t s) {
    static std::mutex mu;
    static std::map<std::pair<int, hipStream_t>, std::unique_ptr<StreamScratch>> pool;
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    auto &e = pool[{dev, s}];
    if (!e) e = std::make_unique<StreamScratch>();
    return *e;
}

// Caller holds b.mu.
static void *scratch_reserve(StreamScratch &b, size_t need) {
    if (b.bytes >= need) return b.ptr;
    size_t sz = std::max<size_t>(need, std::max<size_t>(2 * b.bytes, (size_t)1 << 20));
    void *p = nullptr;
    if (hipMalloc(&p, sz) != hipSuccess) fail(RQC_ENOMEM, "scratch allocation of " + std::to_string(sz) + " bytes failed");
    if (b.ptr) b.retired.push_back(b.ptr);
    b.ptr = p;
    b.bytes = sz;
    return p;
}

} // namespace rqc

using namespace rqc;

struct rqc_circuit {
    Circuit c;
    Network net;
};

struct PendingEvent {
    int cls, op;
    hipEvent_t a, b;
    double flops, bytes, exec_flops;
    int exec_kind;
};

struct rqc_plan : PlanCore {
    int device = 0;
    std::vector<PermDesc> perm_desc;
    // device memory
    std::vector<std::pair<void *, size_t>> owned;
    float2 *d_full = nullptr, *d_leafbuf = nullptr, *d_arena = nullptr;
    LeafSel *d_sel = nullptr;
    SmallStep *d_steps = nullptr;
    SmallTree *d_trees = nullptr;
    double2 *d_acc = nullptr;
    unsigned *d_amax = nullptr;  // operand maxima for the fp16 split scaling
    BitMap *d_smaps = nullptr;   // SM_COUNT maps per streaming op
    BitMap *d_rmaps = nullptr;   // root maps: open index, batched slice index
    PermDesc *d_perm = nullptr;  // permute descriptors
    float2 *d_cache = nullptr;   // global cache: one block per default slice group, plus one spare
    bool cache_filled = false;
    // ordering of calls on one plan across streams: each call waits for the
    // previous call's work (it reuses the arena, leaf buffer, accumulator and
    // global cache) and records its own end
    hipEvent_t done = nullptr;
    bool done_recorded = false;
    // profiling: with opts.profile, the classes whose bit is set get events
    uint32_t prof_mask = 0xFFFFFFFFu;
    rqc_profile_t prof{};
    std::map<std::pair<int, int>, rqc_op_profile_t> op_prof; // (class, program op) -> totals
    std::vector<PendingEvent> pending;
    std::vector<hipEvent_t> pool;

    ~rqc_plan() { release(); }

    void *dalloc(size_t bytes) {
        if (bytes == 0) bytes = 256;
        void *p = nullptr;
        if (opts.alloc) {
            p = opts.alloc(bytes, opts.alloc_ctx);
            if (!p) fail(RQC_ENOMEM, "workspace allocator returned NULL for " + std::to_string(bytes) + " bytes");
        } else {
            hipError_t e = hipMalloc(&p, bytes);
            if (e != hipSuccess) fail(RQC_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        }
        owned.push_back({p, bytes});
        return p;
    }
    void release() {
        for (auto &o : owned) {
            if (opts.alloc) {
                if (opts.free) opts.free(o.first, opts.alloc_ctx);
            } else {
                (void)hipFree(o.first);
            }
        }
        owned.clear();
        if (done) (void)hipEventDestroy(done);
        done = nullptr;
        done_recorded = false;
        for (auto &e : pool) (void)hipEventDestroy(e);
        for (auto &p : pending) (void)hipEventDestroy(p.a), (void)hipEventDestroy(p.b);
        pool.clear();
        pending.clear();
    }
    hipEvent_t ev() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        HIP_OK(hipEventCreate(&e));
        return e;
    }
    void flush_profile() {
        for (auto &p : pending) {
            HIP_OK(hipEventSynchronize(p.b));
            float ms = 0;
            HIP_OK(hipEventElapsedTime(&ms, p.a, p.b));
            prof.launches[p.cls]++;
            prof.seconds[p.cls] += ms * 1e-3;
            prof.flops[p.cls] += p.flops;
            prof.bytes[p.cls] += p.bytes;
            rqc_op_profile_t &o = op_prof[{p.cls, p.op}];
            o.cls = p.cls;
            o.op = p.op;
            o.exec_kind = p.exec_kind;
            o.launches++;
            o.seconds += ms * 1e-3;
            o.flops += p.flops;
            o.bytes += p.bytes;
            o.exec_flops += p.exec_flops;
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pending.clear();
    }
    void upload() {
        const Program &pg = prog;
        for (auto &op : pg.permutes) perm_desc.push_back(make_perm_desc(op.r, op.perm));
        if (opts.dry_run) return;
        try {
            std::vector<float2> f(full.size());
            for (size_t i = 0; i < full.size(); i++) f[i] = make_float2(full[i].real(), full[i].imag());
            d_full = (float2 *)dalloc(f.size() * sizeof(float2));
            d_sel = (LeafSel *)dalloc(sel.size() * sizeof(LeafSel));
            d_leafbuf = (float2 *)dalloc((size_t)pg.leafbuf_elems * sizeof(float2));
            d_arena = (float2 *)dalloc((size_t)std::max<int64_t>(pg.arena_elems, 64) * sizeof(float2));
            d_steps = (SmallStep *)dalloc(std::max<size_t>(1, pg.small_steps.size()) * sizeof(SmallStep));
            d_trees = (SmallTree *)dalloc(std::max<size_t>(1, pg.small_trees.size()) * sizeof(SmallTree));
            d_acc = (double2 *)dalloc(((size_t)1 << spec.open_vars.size()) * sizeof(double2));
            d_amax = (unsigned *)dalloc(256);
            std::vector<BitMap> sm;
            for (auto &so : pg.streams) sm.insert(sm.end(), so.m, so.m + SM_COUNT);
            d_smaps = (BitMap *)dalloc(std::max<size_t>(1, sm.size()) * sizeof(BitMap));
            if (!sm.empty()) HIP_OK(hipMemcpy(d_smaps, sm.data(), sm.size() * sizeof(BitMap), hipMemcpyHostToDevice));
            BitMap rm[2] = {pg.root_open, pg.root_slice};
            d_rmaps = (BitMap *)dalloc(sizeof(rm));
            HIP_OK(hipMemcpy(d_rmaps, rm, sizeof(rm), hipMemcpyHostToDevice));
            d_perm = (PermDesc *)dalloc(std::max<size_t>(1, perm_desc.size()) * sizeof(PermDesc));
            if (!perm_desc.empty())
                HIP_OK(hipMemcpy(d_perm, perm_desc.data(), perm_desc.size() * sizeof(PermDesc), hipMemcpyHostToDevice));
            if (pg.cache && pg.cache_elems > 0)
                d_cache = (float2 *)dalloc((size_t)info.cache_bytes);
            HIP_OK(hipMemcpy(d_full, f.data(), f.size() * sizeof(float2), hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(d_sel, sel.data(), sel.size() * sizeof(LeafSel), hipMemcpyHostToDevice));
            if (!pg.small_steps.empty())
                HIP_OK(hipMemcpy(d_steps, pg.small_steps.data(), pg.small_steps.size() * sizeof(SmallStep),
                                 hipMemcpyHostToDevice));
            if (!pg.small_trees.empty())
                HIP_OK(hipMemcpy(d_trees, pg.small_trees.data(), pg.small_trees.size() * sizeof(SmallTree),
                                 hipMemcpyHostToDevice));
        } catch (...) {
            release();
            throw;
        }
        info.workspace_bytes = 0;
        for (auto &o : owned) info.workspace_bytes += (int64_t)o.second;
    }
};

namespace {

// HIP events around one launch when profiling.  op: the program op (-1 for the
// per-group launches outside the program); xf: flops the launch executes on
// the matrix cores or vector ALUs (kind 0: FP32, 1: bf16/fp16).
struct Timer {
    rqc_plan *p;
    hipStream_t s;
    int cls, op;
    double f, b, xf;
    int xk;
    bool on;
    hipEvent_t a{};
    Timer(rqc_plan *p_, hipStream_t s_, int c, double f_, double b_, int op_ = -1, double xf_ = 0, int xk_ = 0)
        : p(p_), s(s_), cls(c), op(op_), f(f_), b(b_), xf(xf_), xk(xk_) {
        on = p->opts.profile && ((p->prof_mask >> c) & 1u);
        if (on) {
            a = p->ev();
            HIP_OK(hipEventRecord(a, s));
        }
    }
    ~Timer() noexcept(false) {
        if (on) {
            hipEvent_t e = p->ev();
            HIP_OK(hipEventRecord(e, s));
            p->pending.push_back({cls, op, a, e, f, b, xf, xk});
        }
    }
};

template <class F>
rqc_status guard(F &&f) {
    try {
        f();
        return RQC_OK;
    } catch (const Error &e) {
        g_err = e.msg;
        return e.code;
    } catch (const std::bad_alloc &) {
        g_err = "host out of memory";
        return RQC_ENOMEM;
    } catch (const std::exception &e) {
        g_err = e.what();
        return RQC_EINVAL;
    }
}

void dump_plan(const rqc_plan &p) {
    const Program &pg = p.prog;
    std::fprintf(stderr, "plan: %zu fused subtrees (%zu steps, %d LDS elems), %zu ops, arena %lld elems, %lld groups\n",
                 pg.small_trees.size(), pg.small_steps.size(), pg.small_lds_elems, pg.ops.size(),
                 (long long)pg.arena_elems, (long long)p.info.n_groups);
    if (pg.cache)
        std::fprintf(stderr, "  global cache: %lld elements per slice group, %d of %zu fused subtrees independent\n",
                     (long long)pg.cache_elems, pg.n_small_indep, pg.small_trees.size());
    for (const Op &op : pg.ops) {
        if (pg.cache && op.kind != OP_SMALL) std::fprintf(stderr, "%s", op.dep ? "  [per batch]" : "  [cached]");
        if (op.kind == OP_STREAM) {
            const StreamOp &so = pg.streams[op.index];
            // batch legs: r bits that also index B (all of them, and those in a tile)
            int nbat = 0, nbat_tile = 0;
            const BitMap &rb = so.m[SM_RB];
            for (int i = 0; i < rb.n; i++) {
                nbat += rb.len(i);
                const int lo = rb.src(i), hi = rb.src(i) + rb.len(i), L = so.tile_l < 0 ? 0 : so.tile_l;
                nbat_tile += std::max(0, std::min(hi, L) - lo);
            }
            std::fprintf(stderr, "  stream %s rc=%d kc=%d nr=%d nf=%d tile=%d batch=%d/%d flops=%.3g bytes=%.3g\n",
                         so.mx2 ? "mx2" : so.mx ? "mx" : (so.lk ? "lk" : "vec"), so.rc, so.kc, so.nr, so.nf, so.tile_l,
                         nbat_tile, nbat, op.flops, op.bytes);
            if (so.mx || so.lk || so.mx2) {
                // memory bits of A that a tile covers (bit 0 missing = pairs not contiguous)
                for (int which : {SM_EA, SM_EC}) {
                    std::fprintf(stderr, "    tile %s bits:", which == SM_EA ? "A" : "C");
                    const BitMap &e = so.m[which];
                    for (int i = 0; i < e.n; i++)
                        for (int j = 0; j < e.len(i); j++) std::fprintf(stderr, " %d", e.dst(i) + j);
                    std::fprintf(stderr, "\n");
                }
            }
        } else if (op.kind == OP_GEMM) {
            const GemmOp &g = pg.gemms[op.index];
            std::fprintf(stderr, "  gemm b=%lld M=%lld N=%lld K=%lld ak=%d bn=%d ks=%d flops=%.3g\n", (long long)g.batch,
                         (long long)g.M, (long long)g.N, (long long)g.K, g.a_kfast, g.b_nfast, g.ksplit, op.flops);
        } else if (op.kind == OP_PERMUTE) {
            std::fprintf(stderr, "  permute r=%d bytes=%.3g\n", pg.permutes[op.index].r, op.bytes);
        } else {
            std::fprintf(stderr, "  fused subtrees: %zu\n", pg.small_trees.size());
        }
    }
}

// Run the plan's program for every (batch, slice group) pair.
// Slice groups to run: an explicit list of looped-leg values, or 0 .. range-1.
// Slice groups of a call: a list of looped values or the range 0 .. range-1,
// of which the call runs [first, first + count) (cache slots are the absolute
// positions).
struct GroupList {
    const std::vector<uint64_t> *list = nullptr;
    uint64_t range = 0;
    uint64_t first = 0, count = UINT64_MAX;
    uint64_t full() const { return list ? list->size() : range; }
    uint64_t size() const { return first >= full() ? 0 : std::min<uint64_t>(count, full() - first); }
    uint64_t operator[](uint64_t i) const { return list ? (*list)[first + i] : first + i; }
    uint64_t slot(uint64_t i) const { return first + i; }
};

GroupList default_groups(const rqc_plan *p) {
    GroupList g;
    if (p->n_group_range) g.range = p->n_group_range;
    else g.list = &p->groups;
    return g;
}

// Which launches of the program a slice group runs: all of them, only those
// that do not depend on the fixed output bits (filling the global cache), or
// only those that do (reading the filled cache).
enum { RUN_ALL = 0, RUN_INDEP = 1, RUN_DEP = 2 };

// One slice group: leaf selection, then the program's launches for `phase`;
// `slot` picks the group's global-cache block.  Returns the root's address.
float2 *run_group(rqc_plan *p, int phase, const ProjVals &vals, int64_t slot, hipStream_t s) {
    const Program &pg = p->prog;
    float2 *cache = p->d_cache ? p->d_cache + slot * pg.cache_elems : nullptr;
    auto ptr = [&](const Buf &b) -> float2 * {
        return (b.kind == 0 ? p->d_arena : (b.kind == 1 ? p->d_leafbuf : cache)) + b.off;
    };
    {
        Timer t(p, s, RQC_K_LEAF, 0, 16.0 * (double)pg.leafbuf_elems);
        launch_leaf_select(p->d_full, p->d_leafbuf, p->d_sel, (int)p->sel.size(), vals, s);
    }
    for (size_t oi = 0; oi < pg.ops.size(); oi++) {
        const Op &op = pg.ops[oi];
        if (op.kind != OP_SMALL && ((phase == RUN_INDEP && op.dep) || (phase == RUN_DEP && !op.dep))) continue;
        switch (op.kind) {
        case OP_SMALL: {
            const int n = (int)pg.small_trees.size(), ni = pg.n_small_indep;
            const int first = phase == RUN_DEP ? ni : 0, count = phase == RUN_INDEP ? ni : n - first;
            Timer t(p, s, RQC_K_SMALL, op.flops, op.bytes, (int)oi, op.flops, 0);
            launch_small_trees(p->d_steps, p->d_trees + first, count, pg.small_lds_elems, p->d_leafbuf, p->d_arena,
                               cache, s);
            break;
        }
        case OP_STREAM: {
            const StreamOp &so = pg.streams[op.index];
            // the matrix-core forms multiply by B's real block form: 8 real
            // flops per complex multiply-add, as counted; the vector forms the same
            Timer t(p, s, RQC_K_STREAM, op.flops, op.bytes, (int)oi, op.flops, 0);
            launch_stream(so, p->d_smaps + (size_t)op.index * SM_COUNT, ptr(so.a), ptr(so.b), ptr(so.c),
                          so.lk && so.lk_split > 0 ? ptr(so.w) : nullptr, so.mx2 ? ptr(so.b2) : nullptr, s);
            break;
        }
        case OP_PERMUTE: {
            const PermuteOp &po = pg.permutes[op.index];
            Timer t(p, s, RQC_K_PERMUTE, op.flops, op.bytes, (int)oi, 0, 0);
            launch_permute(p->d_perm + op.index, p->perm_desc[op.index].n_tiles, ptr(po.src), ptr(po.dst), s);
            break;
        }
        case OP_GEMM: {
            const GemmOp &go = pg.gemms[op.index];
            GemmArgs ga;
            ga.A = ptr(go.a);
            ga.B = ptr(go.b);
            ga.C = ptr(go.c);
            ga.batch = go.batch;
            ga.M = go.M;
            ga.N = go.N;
            ga.K = go.K;
            ga.sa = go.sa;
            ga.sb = go.sb;
            ga.sc = go.sc;
            ga.a_kfast = go.a_kfast;
            ga.b_nfast = go.b_nfast;
            ga.ksplit = go.ksplit;
            ga.W = go.ksplit > 1 ? ptr(go.w) : nullptr;
            ga.c_ins_pos = go.c_ins_pos;
            ga.c_ins_bits = go.c_ins_bits;
            // executed: three FP32 real products per complex multiply-add, or
            // three bf16/fp16 products of the 2K-long real view per output part
            const bool split = p->opts.precision != RQC_C64 && go.K >= 16;
            Timer t(p, s, RQC_K_GEMM, op.flops, op.bytes, (int)oi, (split ? 3.0 : 0.75) * op.flops, split ? 1 : 0);
            launch_gemm(ga, p->opts.precision, p->d_amax, s);
            break;
        }
        }
    }
    return ptr(pg.root);
}

// Run the plan's program for every (batch, slice group) pair.  `is_default`:
// the groups are the plan's default list (the global cache, if any, holds
// their fixed-bit-independent parts; it is filled on the first such call).
// acc_ext: null = a whole call (zero the plan's accumulator, sum the groups,
// normalise into out_amps / out_f64); else the caller's FP64 accumulator
// [n_batches][2^o], into which the groups' slices are added (overwritten
// first when zero_ext), with no normalisation.
void execute(rqc_plan *p, const GroupList &groups, bool is_default, const uint64_t *fixed_bits, int64_t n_batches,
             void *out_amps, void *out_f64, hipStream_t s, double2 *acc_ext = nullptr, bool zero_ext = false) {
    const Program &pg = p->prog;
    const int n_open = (int)p->spec.open_vars.size();
    const int nl = (int)p->looped.size(), nb = (int)p->batched.size();
    const int64_t nout = (int64_t)1 << n_open;
    const double scale = p->kappa / std::sqrt(p->F);
    const int nfix = (int)p->spec.fixed_vars.size();
    const bool cached = pg.cache && is_default;
    if (!p->done) HIP_OK(hipEventCreateWithFlags(&p->done, hipEventDisableTiming));
    if (p->done_recorded) HIP_OK(hipStreamWaitEvent(s, p->done, 0));
    auto projection = [&](uint64_t fixed, uint64_t g) {
        ProjVals vals{};
        for (int i = 0; i < nfix; i++)
            if ((fixed >> p->spec.fixed_bit[i]) & 1) vals.w[i >> 6] |= 1ull << (i & 63);
        for (int u = 0; u < nl; u++)
            if ((g >> u) & 1) {
                const int idx = nfix + u;
                vals.w[idx >> 6] |= 1ull << (idx & 63);
            }
        return vals;
    };
    if (cached && !p->cache_filled) {
        const GroupList all = default_groups(p);
        for (uint64_t gi = 0; gi < all.size(); gi++) run_group(p, RUN_INDEP, projection(0, all[gi]), (int64_t)gi, s);
        p->cache_filled = true;
    }
    // calls with their own slice list use the spare cache block
    const int64_t spare = p->info.n_groups;
    for (int64_t bi = 0; bi < n_batches; bi++) {
        double2 *acc = acc_ext ? acc_ext + bi * nout : p->d_acc;
        if (!acc_ext || zero_ext) {
            Timer t(p, s, RQC_K_ACCUM, 0, 16.0 * nout);
            launch_zero(acc, nout, s);
        }
        for (uint64_t gi = 0; gi < groups.size(); gi++) {
            const ProjVals vals = projection(fixed_bits[bi], groups[gi]);
            float2 *root = cached ? run_group(p, RUN_DEP, vals, (int64_t)groups.slot(gi), s)
                                  : run_group(p, RUN_ALL, vals, spare, s);
            {
                Timer t(p, s, RQC_K_ACCUM, 0, 8.0 * (double)(nout << nb) + 32.0 * nout);
                launch_accumulate(root, p->d_rmaps, n_open, nb, acc, s);
            }
        }
        if (!acc_ext) {
            Timer t(p, s, RQC_K_FINAL, 0, 16.0 * nout + 8.0 * nout);
            launch_finalize(acc, nout, scale, (float2 *)out_amps + bi * nout,
                            out_f64 ? (double2 *)out_f64 + bi * nout : nullptr, s);
        }
    }
    HIP_OK(hipGetLastError());
    HIP_OK(hipEventRecord(p->done, s));
    p->done_recorded = true;
    if (p->opts.profile && p->pending.size() > 8192) p->flush_profile();
}

// Device time of one batch on a candidate tree (after one warm-up batch, which
// also fills a global cache), in seconds.
double time_candidate(const PlanCore &base, const PlanCore::Candidate &cand) {
    auto Q = std::make_unique<rqc_plan>();
    rqc_plan &q = *Q;
    q.opts = base.opts;
    q.opts.profile = 0;
    q.opts.autotune = 0;
    q.spec = base.spec;
    q.tree = cand.tree;
    q.sliced = cand.sliced;
    q.user_legs = base.user_legs;
    HIP_OK(hipGetDevice(&q.device));
    plan_finish(q);
    q.upload();
    const int64_t nout = (int64_t)1 << q.spec.open_vars.size();
    float2 *amps = (float2 *)q.dalloc((size_t)nout * sizeof(float2));
    struct Res {
        hipStream_t s = nullptr;
        hipEvent_t a = nullptr, b = nullptr;
        ~Res() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
            if (s) (void)hipStreamDestroy(s);
        }
    } r;
    HIP_OK(hipStreamCreate(&r.s)); // default priority
    HIP_OK(hipEventCreate(&r.a));
    HIP_OK(hipEventCreate(&r.b));
    const uint64_t zero = 0;
    execute(&q, default_groups(&q), true, &zero, 1, amps, nullptr, r.s);
    HIP_OK(hipEventRecord(r.a, r.s));
    execute(&q, default_groups(&q), true, &zero, 1, amps, nullptr, r.s);
    HIP_OK(hipEventRecord(r.b, r.s));
    HIP_OK(hipEventSynchronize(r.b));
    float ms = 0;
    HIP_OK(hipEventElapsedTime(&ms, r.a, r.b));
    return 1e-3 * ms;
}

// R[i] = ||psi_i||^2 by contracting the doubled network on the GPU (Fig. 1).
std::vector<double> gpu_norms(const rqc_plan_opts &outer, const NetSpec &spec, const std::vector<int> &S) {
    auto P = std::make_unique<rqc_plan>();
    rqc_plan &q = *P;
    q.opts = rqc_plan_opts{};
    q.opts.max_log2_tensor = 28;
    q.opts.n_sliced_target = -1;
    q.opts.max_log2_batched = 28;
    q.opts.path_trials = 32;
    q.opts.path_seed = outer.path_seed;
    q.opts.alloc = outer.alloc;
    q.opts.free = outer.free;
    q.opts.alloc_ctx = outer.alloc_ctx;
    q.spec = spec;
    q.info.n_qubits = 0;
    plan_tree(q, nullptr, 0, nullptr);
    plan_finish(q);
    HIP_OK(hipGetDevice(&q.device));
    q.upload();
    const size_t n = (size_t)1 << S.size();
    // output buffers from the norm plan's workspace (the caller's allocator
    // when one is given), released with that plan
    float2 *amps = (float2 *)q.dalloc(n * sizeof(float2));
    double2 *r64 = (double2 *)q.dalloc(n * sizeof(double2));
    std::vector<double2> host(n);
    uint64_t zero = 0;
    execute(&q, default_groups(&q), true, &zero, 1, amps, r64, nullptr);
    HIP_OK(hipMemcpy(host.data(), r64, n * sizeof(double2), hipMemcpyDeviceToHost));
    HIP_OK(hipStreamSynchronize(nullptr));
    std::vector<double> R(n);
    for (size_t i = 0; i < n; i++) R[i] = host[i].x;
    return R;
}

} // namespace

extern "C" {

const char *rqc_last_error(void) { return g_err.c_str(); }
const char *rqc_version(void) { return "librqc 0.2 (gfx950)"; }

rqc_status rqc_load_circuit(const char *text, size_t len, rqc_circuit **out) {
    return guard([&] {
        if (!text || !out) fail(RQC_EINVAL, "null argument");
        auto c = std::make_unique<rqc_circuit>();
        c->c = parse_circuit(text, len);
        c->net = build_network(c->c);
        *out = c.release();
    });
}

rqc_status rqc_circuit_info(const rqc_circuit *c, int32_t *n_qubits, int32_t *n_variables, int32_t *n_gates) {
    return guard([&] {
        if (!c) fail(RQC_EINVAL, "null circuit");
        if (n_qubits) *n_qubits = c->c.n;
        if (n_variables) *n_variables = c->net.n_vars;
        if (n_gates) *n_gates = (int32_t)c->c.gates.size();
    });
}

void rqc_circuit_destroy(rqc_circuit *c) { delete c; }

rqc_status rqc_plan_create(const rqc_circuit *c, const int32_t *path, int32_t n_path_pairs,
                           const int32_t *sliced_legs, int32_t n_sliced, const int32_t *open_qubits,
                           int32_t n_open, const rqc_plan_opts *opts, rqc_plan **out) {
    return guard([&] {
        if (!c || !out) fail(RQC_EINVAL, "null argument");
        if (n_open < 0 || n_open > c->c.n || (n_open > 0 && !open_qubits)) fail(RQC_EINVAL, "bad open qubits");
        if (n_open > 30) fail(RQC_EINVAL, "at most 30 open qubits");
        if (n_sliced < 0 || n_path_pairs < 0) fail(RQC_EINVAL, "negative count");
        auto t0 = std::chrono::steady_clock::now();
        auto P = std::make_unique<rqc_plan>();
        rqc_plan &p = *P;
        if (opts) p.opts = *opts;
        if (p.opts.max_log2_batched <= 0) p.opts.max_log2_batched = 28;
        if (p.opts.precision < 0 || p.opts.precision > 2) fail(RQC_EINVAL, "unknown precision");
        const double f = p.opts.target_fidelity;
        const bool partial = f > 0 && f < 1;

        if (!p.opts.dry_run) {
            check_device();
            HIP_OK(hipGetDevice(&p.device));
        }
        std::vector<int> oq(open_qubits, open_qubits + n_open);
        p.spec = circuit_spec(c->net, oq);
        p.info.n_qubits = c->c.n;
        std::vector<int> user;
        if (sliced_legs) user.assign(sliced_legs, sliced_legs + n_sliced);
        std::unique_ptr<LightCones> lc;
        if (partial && !path && !sliced_legs) lc = std::make_unique<LightCones>(light_cones(c->net));
        plan_tree(p, path, n_path_pairs, sliced_legs ? &user : nullptr, lc.get());
        // time the best candidates on the device (skipping any estimated over
        // 2 s); another tree replaces the estimate's choice only if it is at
        // least 5 % faster, so that timing noise does not change the plan
        if (p.opts.autotune > 1 && !partial && !p.opts.dry_run && !path && p.candidates.size() > 1 &&
            p.candidates[0].est <= 2.0) {
            size_t best = 0;
            double best_t = 0.95 * time_candidate(p, p.candidates[0]);
            for (size_t i = 1; i < p.candidates.size() && (int)i < p.opts.autotune; i++) {
                if (p.candidates[i].est > 2.0) continue;
                const double t = time_candidate(p, p.candidates[i]);
                if (t < best_t) best_t = t, best = i;
            }
            p.tree = p.candidates[best].tree;
            p.sliced = p.candidates[best].sliced;
        }
        if (partial && p.opts.dry_run) {
            // the norms need the GPU: a host-only plan selects S and stops there
            p.S = sliced_vertex_select(light_cones(c->net), p.sliced, partial_k0(p.opts));
            p.F = 0;
        } else if (partial) {
            rqc_plan_opts o = p.opts;
            plan_partial(p, c->net, [&](const NetSpec &ds, const std::vector<int> &S) { return gpu_norms(o, ds, S); });
        }
        plan_finish(p);
        if (const char *d = std::getenv("RQC_DUMP_PLAN"); d && d[0] == '1') dump_plan(p);
        p.upload();
        p.info.plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *out = P.release();
    });
}

rqc_status rqc_plan_info(const rqc_plan *p, rqc_plan_info_t *info) {
    return guard([&] {
        if (!p || !info) fail(RQC_EINVAL, "null argument");
        *info = p->info;
    });
}

rqc_status rqc_plan_sliced_legs(const rqc_plan *p, int32_t *legs, int32_t cap, int32_t *count) {
    return guard([&] {
        if (!p) fail(RQC_EINVAL, "null plan");
        if (count) *count = (int32_t)p->sliced.size();
        for (size_t i = 0; legs && i < p->sliced.size() && (int32_t)i < cap; i++) legs[i] = p->sliced[i];
    });
}

rqc_status rqc_plan_path(const rqc_plan *p, int32_t *pairs, int32_t cap, int32_t *count) {
    return guard([&] {
        if (!p) fail(RQC_EINVAL, "null plan");
        if (count) *count = (int32_t)p->tree.steps.size();
        for (size_t s = 0; pairs && s < p->tree.steps.size() && (int32_t)s < cap; s++) {
            pairs[2 * s] = p->tree.steps[s].first;
            pairs[2 * s + 1] = p->tree.steps[s].second;
        }
    });
}

rqc_status rqc_plan_describe(const rqc_plan *p, char *buf, size_t cap, size_t *len) {
    return guard([&] {
        if (!p) fail(RQC_EINVAL, "null plan");
        const std::string d = describe_program(*p);
        if (len) *len = d.size() + 1;
        if (buf && cap > 0) {
            const size_t n = std::min(cap - 1, d.size());
            std::memcpy(buf, d.data(), n);
            buf[n] = 0;
        }
    });
}

rqc_status rqc_plan_partial(const rqc_plan *p, int32_t *S, int32_t capS, uint64_t *X, int64_t capX, double *R,
                            int64_t capR) {
    return guard([&] {
        if (!p) fail(RQC_EINVAL, "null plan");
        for (size_t i = 0; S && i < p->S.size() && (int64_t)i < capS; i++) S[i] = p->S[i];
        for (size_t i = 0; X && i < p->X.size() && (int64_t)i < capX; i++) X[i] = p->X[i];
        for (size_t i = 0; R && i < p->R.size() && (int64_t)i < capR; i++) R[i] = p->R[i];
    });
}

rqc_status rqc_plan_slices(const rqc_plan *p, uint64_t *ids, int64_t cap, int64_t *count) {
    return guard([&] {
        if (!p || !count) fail(RQC_EINVAL, "null argument");
        GroupList g = default_groups(p);
        const int nb = (int)p->batched.size(), nl = (int)p->looped.size();
        const double total = (double)g.size() * std::exp2((double)nb);
        if (total > 9e18) fail(RQC_EINVAL, "slice list too long");
        *count = (int64_t)g.size() << nb;
        int64_t k = 0;
        for (uint64_t gi = 0; gi < g.size() && k < cap && ids; gi++)
            for (uint64_t b = 0; b < ((uint64_t)1 << nb) && k < cap; b++) {
                uint64_t sid = 0;
                const uint64_t lv = g[gi];
                for (int u = 0; u < nl; u++) sid |= ((lv >> u) & 1) << p->looped_bit[u];
                for (int u = 0; u < nb; u++) sid |= ((b >> u) & 1) << p->batched_bit[u];
                ids[k++] = sid;
            }
    });
}

rqc_status rqc_plan_profile(const rqc_plan *pc, rqc_profile_t *out) {
    return guard([&] {
        if (!pc || !out) fail(RQC_EINVAL, "null argument");
        rqc_plan *p = const_cast<rqc_plan *>(pc);
        p->flush_profile();
        *out = p->prof;
    });
}

rqc_status rqc_plan_profile_reset(rqc_plan *p) {
    return guard([&] {
        if (!p) fail(RQC_EINVAL, "null plan");
        p->flush_profile();
        p->prof = rqc_profile_t{};
        p->op_prof.clear();
    });
}

rqc_status rqc_plan_profile_classes(rqc_plan *p, uint32_t mask) {
    return guard([&] {
        if (!p) fail(RQC_EINVAL, "null plan");
        if (mask >> RQC_K_CLASSES) fail(RQC_EINVAL, "unknown kernel class in the mask");
        p->prof_mask = mask;
    });
}

rqc_status rqc_plan_profile_ops(const rqc_plan *pc, rqc_op_profile_t *ops, int32_t cap, int32_t *count) {
    return guard([&] {
        if (!pc || !count) fail(RQC_EINVAL, "null argument");
        rqc_plan *p = const_cast<rqc_plan *>(pc);
        p->flush_profile();
        *count = (int32_t)p->op_prof.size();
        int32_t k = 0;
        for (auto &kv : p->op_prof) {
            if (!ops || k >= cap) break;
            ops[k++] = kv.second;
        }
    });
}

void rqc_plan_destroy(rqc_plan *p) {
    if (!p) return;
    // with the library's own hipMalloc workspace, wait for the device before
    // freeing; a caller-supplied allocator owns that ordering
    if (!p->opts.dry_run && !p->opts.alloc) (void)hipDeviceSynchronize();
    delete p;
}

rqc_status rqc_contract_amplitudes(rqc_plan *p, const uint64_t *slice_ids, int64_t n_slices,
                                   const uint64_t *fixed_bits, int64_t n_batches, void *out_amps, void *out_f64,
                                   void *hip_stream) {
    return guard([&] {
        if (!p) fail(RQC_EINVAL, "null plan");
        if (p->opts.dry_run) fail(RQC_EINVAL, "a dry-run plan cannot be executed");
        if (n_batches < 0) fail(RQC_EINVAL, "negative batch count");
        if (n_batches == 0) return;
        if (!fixed_bits || !out_amps) fail(RQC_EINVAL, "null fixed_bits or out_amps");
        int dev = 0;
        HIP_OK(hipGetDevice(&dev));
        if (dev != p->device) fail(RQC_EDEVICE, "plan belongs to another device");
        const int nl = (int)p->looped.size(), nb = (int)p->batched.size();
        if (!slice_ids) {
            execute(p, default_groups(p), true, fixed_bits, n_batches, out_amps, out_f64, (hipStream_t)hip_stream);
            return;
        }
        if (n_slices < 0) fail(RQC_EINVAL, "negative slice count");
        std::vector<std::pair<uint64_t, uint64_t>> kv; // (looped value, batched value)
        for (int64_t i = 0; i < n_slices; i++) {
            const uint64_t sid = slice_ids[i];
            if (p->sliced.size() < 64 && (sid >> p->sliced.size()))
                fail(RQC_EINVAL, "slice id has bits beyond the sliced legs");
            uint64_t lv = 0, bv = 0;
            for (int u = 0; u < nl; u++) lv |= ((sid >> p->looped_bit[u]) & 1) << u;
            for (int u = 0; u < nb; u++) bv |= ((sid >> p->batched_bit[u]) & 1) << u;
            kv.push_back({lv, bv});
        }
        std::sort(kv.begin(), kv.end());
        std::vector<uint64_t> groups;
        for (size_t i = 0; i < kv.size();) {
            size_t j = i;
            while (j < kv.size() && kv[j].first == kv[i].first) j++;
            if (j - i != ((size_t)1 << nb))
                fail(RQC_EINVAL, "slice list must contain whole batched groups (" + std::to_string((size_t)1 << nb) +
                                     " slices per looped value)");
            for (size_t k = i; k < j; k++)
                if (kv[k].second != (uint64_t)(k - i)) fail(RQC_EINVAL, "repeated slice id");
            groups.push_back(kv[i].first);
            i = j;
        }
        GroupList gl;
        gl.list = &groups;
        execute(p, gl, false, fixed_bits, n_batches, out_amps, out_f64, (hipStream_t)hip_stream);
    });
}

rqc_status rqc_contract_groups(rqc_plan *p, int64_t first_group, int64_t n_groups, const uint64_t *fixed_bits,
                               int64_t n_batches, void *acc_f64, void *hip_stream) {
    return guard([&] {
        if (!p) fail(RQC_EINVAL, "null plan");
        if (p->opts.dry_run) fail(RQC_EINVAL, "a dry-run plan cannot be executed");
        if (n_batches < 0 || first_group < 0 || n_groups < 0) fail(RQC_EINVAL, "negative count");
        GroupList gl = default_groups(p);
        if ((uint64_t)first_group > gl.full() || (uint64_t)n_groups > gl.full() - (uint64_t)first_group)
            fail(RQC_EINVAL, "group range beyond the plan's default slice list");
        if (n_batches == 0) return;
        if (!fixed_bits || !acc_f64) fail(RQC_EINVAL, "null fixed_bits or accumulator");
        int dev = 0;
        HIP_OK(hipGetDevice(&dev));
        if (dev != p->device) fail(RQC_EDEVICE, "plan belongs to another device");
        gl.first = (uint64_t)first_group;
        gl.count = (uint64_t)n_groups;
        execute(p, gl, true, fixed_bits, n_batches, nullptr, nullptr, (hipStream_t)hip_stream, (double2 *)acc_f64,
                first_group == 0);
    });
}

rqc_status rqc_finalize_amplitudes(rqc_plan *p, const void *acc_f64, int64_t n_batches, void *out_amps,
                                   void *out_f64, void *hip_stream) {
    return guard([&] {
        if (!p) fail(RQC_EINVAL, "null plan");
        if (p->opts.dry_run) fail(RQC_EINVAL, "a dry-run plan cannot be executed");
        if (n_batches < 0) fail(RQC_EINVAL, "negative batch count");
        if (n_batches == 0) return;
        if (!acc_f64 || !out_amps) fail(RQC_EINVAL, "null accumulator or out_amps");
        hipStream_t s = (hipStream_t)hip_stream;
        const int64_t nout = (int64_t)1 << p->spec.open_vars.size();
        const double scale = p->kappa / std::sqrt(p->F);
        // ordered after the plan's previous calls (the accumulator they filled)
        if (p->done_recorded) HIP_OK(hipStreamWaitEvent(s, p->done, 0));
        for (int64_t bi = 0; bi < n_batches; bi++) {
            Timer t(p, s, RQC_K_FINAL, 0, 16.0 * nout + 8.0 * nout);
            launch_finalize((const double2 *)acc_f64 + bi * nout, nout, scale, (float2 *)out_amps + bi * nout,
                            out_f64 ? (double2 *)out_f64 + bi * nout : nullptr, s);
        }
        HIP_OK(hipGetLastError());
        if (!p->done) HIP_OK(hipEventCreateWithFlags(&p->done, hipEventDisableTiming));
        HIP_OK(hipEventRecord(p->done, s));
        p->done_recorded = true;
    });
}

// Argument checks shared by the two sampling entry points; returns the number
// of sampled items (sub-batches, or steps in pick mode).
static int64_t check_sample_args(const void *amps, const uint64_t *fixed_bits, int64_t n_batches,
                                 const int32_t *open_qubits, int32_t n_open, int32_t log2_NA, int32_t n_qubits,
                                 double alpha, double F_norm, int64_t pick_steps, int64_t n_samples,
                                 const uint64_t *out_samples, const int64_t *n_out) {
    if (!amps || !n_out || (n_samples > 0 && !out_samples)) fail(RQC_EINVAL, "null argument");
    if (n_qubits < 1 || n_qubits > 64) fail(RQC_EINVAL, "n_qubits must be 1..64");
    if (n_open < 0 || n_open > n_qubits || n_open > 30 || (n_open > 0 && !open_qubits))
        fail(RQC_EINVAL, "bad open qubits");
    if (log2_NA < 0 || log2_NA > n_open) fail(RQC_EINVAL, "log2_NA must be within the open batch");
    if (!(alpha > 0) || !(F_norm > 0)) fail(RQC_EINVAL, "alpha and F_norm must be positive");
    if (n_samples < 0 || n_batches < 0 || pick_steps < 0) fail(RQC_EINVAL, "negative count");
    if (pick_steps > 0 && (n_batches != 1 || n_open != n_qubits))
        fail(RQC_EINVAL, "pick mode needs one batch with every qubit open");
    if (n_batches > 0 && !fixed_bits) fail(RQC_EINVAL, "null fixed_bits");
    for (int b = 0; b < n_open; b++)
        if (open_qubits[b] < 0 || open_qubits[b] >= n_qubits) fail(RQC_EINVAL, "open qubit out of range");
    if (pick_steps == 0 && n_batches > ((int64_t)1 << 40)) fail(RQC_EINVAL, "too many batches");
    return pick_steps > 0 ? pick_steps : n_batches * ((int64_t)1 << (n_open - log2_NA));
}

rqc_status rqc_rejection_sample(const void *amps, const uint64_t *fixed_bits, int64_t n_batches,
                                const int32_t *open_qubits, int32_t n_open, int32_t log2_NA, int32_t n_qubits,
                                double alpha, double F_norm, uint64_t seed, uint64_t batch_index_base,
                                int64_t pick_steps, int64_t n_samples, uint64_t *out_samples, int64_t *n_out,
                                rqc_sample_stats *stats, void *hip_stream) {
    rqc_status st = guard([&] {
        const int64_t items = check_sample_args(amps, fixed_bits, n_batches, open_qubits, n_open, log2_NA, n_qubits,
                                                alpha, F_norm, pick_steps, n_samples, out_samples, n_out);
        hipStream_t s = (hipStream_t)hip_stream;
        StreamScratch &sc = stream_scratch(s);
        std::lock_guard<std::mutex> lk(sc.mu);
        void *w = scratch_reserve(sc, sampler_scratch_bytes(items, n_batches, n_open));
        const hipError_t e = run_sampler((const float2 *)amps, fixed_bits, n_batches, open_qubits, n_open, log2_NA,
                                         n_qubits, alpha, F_norm, seed, batch_index_base, pick_steps, n_samples,
                                         out_samples, n_out, stats, w, s);
        if (e != hipSuccess) fail(RQC_EDEVICE, std::string("sampler: ") + hipGetErrorString(e));
    });
    if (st == RQC_OK && *n_out < n_samples) {
        g_err = "fewer accepted samples than requested";
        return RQC_ESHORT;
    }
    return st;
}

rqc_status rqc_rejection_sample_static(const void *amps, const uint64_t *fixed_bits, int64_t n_batches,
                                       const int32_t *open_qubits, int32_t n_open, int32_t log2_NA,
                                       int32_t n_qubits, double alpha, double F_norm, uint64_t seed,
                                       uint64_t batch_index_base, int64_t pick_steps, int64_t n_samples,
                                       uint64_t *out_samples, int64_t *n_out, rqc_sample_stats *stats,
                                       void *hip_stream) {
    rqc_status st = guard([&] {
        const int64_t items = check_sample_args(amps, fixed_bits, n_batches, open_qubits, n_open, log2_NA, n_qubits,
                                                alpha, F_norm, pick_steps, n_samples, out_samples, n_out);
        const size_t need = sampler_scratch_bytes(items, n_batches, n_open);
        if (need > (size_t)RQC_SAMPLE_STATIC_SCRATCH_BYTES)
            fail(RQC_EINVAL, "the call needs " + std::to_string(need) + " bytes of scratch; the fixed array holds " +
                                 std::to_string((size_t)RQC_SAMPLE_STATIC_SCRATCH_BYTES));
        void *w = nullptr;
        std::mutex *call_mu = nullptr;
        HIP_OK(static_scratch(&w, &call_mu));
        // one call at a time per device: the array is shared, and each call has
        // finished with it (the sampler synchronises its stream) when it returns
        std::lock_guard<std::mutex> lk(*call_mu);
        const hipError_t e = run_sampler((const float2 *)amps, fixed_bits, n_batches, open_qubits, n_open, log2_NA,
                                         n_qubits, alpha, F_norm, seed, batch_index_base, pick_steps, n_samples,
                                         out_samples, n_out, stats, w, (hipStream_t)hip_stream);
        if (e != hipSuccess) fail(RQC_EDEVICE, std::string("sampler: ") + hipGetErrorString(e));
    });
    if (st == RQC_OK && *n_out < n_samples) {
        g_err = "fewer accepted samples than requested";
        return RQC_ESHORT;
    }
    return st;
}

rqc_status rqc_select_top(const void *amps, uint64_t fixed_bits, const int32_t *open_qubits, int32_t n_open,
                          int32_t n_qubits, int64_t count, uint64_t *out_samples, void *hip_stream) {
    return guard([&] {
        if (!amps || (count > 0 && !out_samples)) fail(RQC_EINVAL, "null argument");
        if (n_qubits < 1 || n_qubits > 64) fail(RQC_EINVAL, "n_qubits must be 1..64");
        if (n_open < 0 || n_open > n_qubits || n_open > 30 || (n_open > 0 && !open_qubits))
            fail(RQC_EINVAL, "bad open qubits");
        uint64_t seen = 0;
        for (int b = 0; b < n_open; b++) {
            if (open_qubits[b] < 0 || open_qubits[b] >= n_qubits) fail(RQC_EINVAL, "open qubit out of range");
            if ((seen >> open_qubits[b]) & 1) fail(RQC_EINVAL, "open qubit repeated");
            seen |= 1ull << open_qubits[b];
        }
        if (count < 0 || count > ((int64_t)1 << n_open)) fail(RQC_EINVAL, "count must be within the batch");
        if (count == 0) return;
        check_device();
        hipStream_t s = (hipStream_t)hip_stream;
        StreamScratch &sc = stream_scratch(s);
        std::lock_guard<std::mutex> lk(sc.mu);
        // stream order keeps later calls on s off this block until these
        // kernels are done; other streams have blocks of their own
        void *w = scratch_reserve(sc, select_scratch_bytes((int64_t)1 << n_open));
        launch_select_top((const float2 *)amps, n_open, open_qubits, fixed_bits, count, out_samples, w, s);
        HIP_OK(hipGetLastError());
    });
}

rqc_status rqc_prob_sums(const void *amps, int64_t n_rows, int64_t row_len, int32_t n_qubits, double *sums,
                         double *xeb, void *hip_stream) {
    return guard([&] {
        if (n_rows < 0 || row_len < 0) fail(RQC_EINVAL, "negative size");
        if (n_rows == 0) return;
        if (!sums || (row_len > 0 && !amps)) fail(RQC_EINVAL, "null argument");
        if (xeb && (row_len == 0 || n_qubits < 1 || n_qubits > 64))
            fail(RQC_EINVAL, "the XEB needs row_len >= 1 and n_qubits in 1..64");
        const int64_t nchunk = (row_len + 8191) / 8192;
        if (n_rows >= ((int64_t)1 << 31) || n_rows * nchunk >= ((int64_t)1 << 31))
            fail(RQC_EINVAL, "too many rows or chunks for one launch");
        check_device();
        hipStream_t s = (hipStream_t)hip_stream;
        StreamScratch &sc = stream_scratch(s);
        std::lock_guard<std::mutex> lk(sc.mu);
        void *w = scratch_reserve(sc, prob_sums_scratch_bytes(n_rows, row_len));
        launch_prob_sums((const float2 *)amps, n_rows, row_len, n_qubits, sums, xeb, w, s);
        HIP_OK(hipGetLastError());
    });
}

rqc_status rqc_kernel_cgemm(const void *A, const void *B, void *C, int64_t batch, int64_t M, int64_t N, int64_t K,
                            int32_t a_kfast, int32_t b_nfast, int32_t precision, void *hip_stream) {
    return guard([&] {
        if (!A || !B || !C) fail(RQC_EINVAL, "null operand");
        auto pow2 = [](int64_t x) { return x > 0 && (x & (x - 1)) == 0; };
        if (batch < 1 || !pow2(M) || !pow2(N) || !pow2(K) || M < 64 || N < 64 || K < 8)
            fail(RQC_EINVAL, "GEMM needs powers of two with M, N >= 64 and K >= 8");
        if (batch * M * N >= ((int64_t)1 << 34)) fail(RQC_EINVAL, "GEMM output too large");
        if (precision < 0 || precision > 2) fail(RQC_EINVAL, "unknown precision");
        check_device();
        GemmArgs g;
        g.A = (const float2 *)A;
        g.B = (const float2 *)B;
        g.C = (float2 *)C;
        g.batch = batch;
        g.M = M;
        g.N = N;
        g.K = K;
        g.sa = M * K;
        g.sb = K * N;
        g.sc = M * N;
        g.a_kfast = a_kfast ? 1 : 0;
        g.b_nfast = b_nfast ? 1 : 0;
        hipStream_t s = (hipStream_t)hip_stream;
        // the fp16 scaling maxima: two words of this stream's scratch, written
        // and read in stream order
        StreamScratch &sc = stream_scratch(s);
        std::lock_guard<std::mutex> lk(sc.mu);
        launch_gemm(g, precision, (unsigned *)scratch_reserve(sc, 256), s);
        HIP_OK(hipGetLastError());
    });
}

rqc_status rqc_kernel_permute(const void *src, void *dst, int32_t r, const int32_t *perm, void *hip_stream) {
    return guard([&] {
        if (!src || !dst || !perm) fail(RQC_EINVAL, "null argument");
        if (r < 0 || r > 34) fail(RQC_EINVAL, "rank must be 0..34");
        std::vector<int> pv(r);
        std::vector<char> seen(r, 0);
        for (int i = 0; i < r; i++) {
            if (perm[i] < 0 || perm[i] >= r || seen[perm[i]]) fail(RQC_EINVAL, "perm is not a permutation");
            seen[perm[i]] = 1;
            pv[i] = perm[i];
        }
        check_device();
        PermDesc d = make_perm_desc(r, pv);
        // the descriptor travels in the kernel arguments
        launch_permute_value(d, (const float2 *)src, (float2 *)dst, (hipStream_t)hip_stream);
        HIP_OK(hipGetLastError());
    });
}

} // extern "C"
