// C-ABI of librqc: circuit handles, planning, the slice-group executor and the
// sampler entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <memory>
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

// Planning helpers declared in lower.cpp
Program lower_tree(const Tree &tree, const std::vector<Legs> &legs, const std::vector<int> &leaf_offsets,
                   std::vector<int> &root_layout);

static void check_device() {
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_OK(hipGetDeviceProperties(&prop, dev));
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        fail(RQC_EDEVICE, std::string("librqc is built for gfx950; current device is ") + prop.gcnArchName);
}

} // namespace rqc

using namespace rqc;

struct rqc_circuit {
    Circuit c;
    Network net;
};

struct PendingEvent {
    int cls;
    hipEvent_t a, b;
    double flops, bytes;
};

struct rqc_plan {
    int device = 0;
    rqc_plan_opts opts{};
    Network net;
    Tree tree;
    std::vector<int> open_qubits;
    std::vector<int> sliced, batched, looped; // variable ids
    std::vector<int> looped_bit, batched_bit; // bit position of each in a slice id
    // partial slicing
    std::vector<int> S;
    std::vector<int> S_bit;                   // bit position of S members in a slice id
    std::vector<uint64_t> X;
    std::vector<double> R;
    double F = 1.0;
    // projected variables: fixed output qubits first, then looped legs
    std::vector<int> fixed_qubit;
    Program prog;
    std::vector<PermDesc> perm_desc;
    rqc_plan_info_t info{};
    // device memory
    std::vector<std::pair<void *, size_t>> owned;
    float2 *d_full = nullptr, *d_leafbuf = nullptr, *d_arena = nullptr;
    LeafSel *d_sel = nullptr;
    SmallStep *d_steps = nullptr;
    SmallTree *d_trees = nullptr;
    double2 *d_acc = nullptr;
    int n_leaves = 0;
    // profiling
    rqc_profile_t prof{};
    std::vector<PendingEvent> pending;
    std::vector<hipEvent_t> pool;

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
            pool.push_back(p.a);
            pool.push_back(p.b);
        }
        pending.clear();
    }
};

namespace {

struct Timer {
    rqc_plan *p;
    hipStream_t s;
    int cls;
    double f, b;
    hipEvent_t a{};
    Timer(rqc_plan *p_, hipStream_t s_, int c, double f_, double b_) : p(p_), s(s_), cls(c), f(f_), b(b_) {
        if (p->opts.profile) {
            a = p->ev();
            HIP_OK(hipEventRecord(a, s));
        }
    }
    ~Timer() noexcept(false) {
        if (p->opts.profile) {
            hipEvent_t e = p->ev();
            HIP_OK(hipEventRecord(e, s));
            p->pending.push_back({cls, a, e, f, b});
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

std::vector<Legs> leaf_leg_sets(const Network &net) {
    std::vector<Legs> out;
    for (auto &L : net.leaves) {
        Legs l(L.legs);
        std::sort(l.begin(), l.end());
        out.push_back(l);
    }
    return out;
}

} // namespace

extern "C" {

const char *rqc_last_error(void) { return g_err.c_str(); }
const char *rqc_version(void) { return "librqc 0.1 (gfx950)"; }

rqc_status rqc_load_circuit(const char *text, size_t len, rqc_circuit **out) {
    return guard([&] {
        if (!text || !out) fail(RQC_EINVAL, "null argument");
        auto *c = new rqc_circuit;
        try {
            c->c = parse_circuit(text, len);
            c->net = build_network(c->c);
        } catch (...) {
            delete c;
            throw;
        }
        *out = c;
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
        auto t0 = std::chrono::steady_clock::now();
        auto P = std::make_unique<rqc_plan>();
        rqc_plan &p = *P;
        if (opts) p.opts = *opts;
        if (p.opts.max_log2_batched <= 0) p.opts.max_log2_batched = 28;
        if (p.opts.precision < 0 || p.opts.precision > 2) fail(RQC_EINVAL, "unknown precision");
        if (!p.opts.dry_run) {
            check_device();
            HIP_OK(hipGetDevice(&p.device));
        }
        p.net = c->net;
        const Network &net = p.net;
        const int n = net.n_qubits, nv = net.n_vars;
        std::vector<char> is_open(n, 0);
        for (int b = 0; b < n_open; b++) {
            int q = open_qubits[b];
            if (q < 0 || q >= n || is_open[q]) fail(RQC_EINVAL, "open qubits must be distinct and in range");
            is_open[q] = 1;
            p.open_qubits.push_back(q);
        }
        std::vector<char> kept(nv, 0), fixed_out(nv, 0), forbidden(nv, 0);
        for (int v = 0; v < n && v < nv; v++) forbidden[v] = 1;
        for (int q = 0; q < n; q++) {
            forbidden[net.out_var[q]] = 1;
            if (is_open[q]) kept[net.out_var[q]] = 1;
            else fixed_out[net.out_var[q]] = 1;
        }
        std::vector<Legs> leaf_legs = leaf_leg_sets(net);
        std::vector<Legs> path_legs(leaf_legs.size());
        for (size_t i = 0; i < leaf_legs.size(); i++)
            for (int v : leaf_legs[i])
                if (!fixed_out[v]) path_legs[i].push_back(v);
        // -------- contraction tree and sliced legs
        std::vector<char> none(nv, 0);
        std::vector<int> user_sliced;
        if (sliced_legs) {
            std::vector<char> seen(nv, 0);
            for (int i = 0; i < n_sliced; i++) {
                int v = sliced_legs[i];
                if (v < 0 || v >= nv || forbidden[v] || seen[v])
                    fail(RQC_EINVAL, "sliced leg " + std::to_string(v) + " is not an internal variable");
                seen[v] = 1;
                user_sliced.push_back(v);
            }
        }
        if (path) {
            Tree t;
            t.n_leaves = (int)leaf_legs.size();
            std::vector<char> used(t.n_leaves + n_path_pairs, 0);
            for (int s = 0; s < n_path_pairs; s++) {
                int a = path[2 * s], b = path[2 * s + 1];
                int lim = t.n_leaves + s;
                if (a < 0 || b < 0 || a >= lim || b >= lim || a == b || used[a] || used[b])
                    fail(RQC_EINVAL, "path pair " + std::to_string(s) + " is not a valid SSA pair");
                used[a] = used[b] = 1;
                t.steps.push_back({a, b});
            }
            if (n_path_pairs != t.n_leaves - 1) fail(RQC_EINVAL, "path must contract all tensors into one");
            p.tree = t;
            if (!sliced_legs) {
                auto legs = tree_legs(t, path_legs, nv, fixed_out, kept);
                p.sliced = greedy_slice(t, legs, nv, forbidden, p.opts.max_log2_tensor, p.opts.n_sliced_target);
            } else {
                p.sliced = user_sliced;
            }
        } else {
            int trials = p.opts.path_trials > 0 ? p.opts.path_trials : 16;
            double best = 1e300;
            for (int tr = 0; tr < trials; tr++) {
                double temp = tr == 0 ? 0.0 : 0.1 + 0.9 * (double)(tr % 8) / 8.0;
                Tree t = greedy_tree(path_legs, nv, kept, p.opts.path_seed * 1000003ull + (uint64_t)tr, temp);
                auto legs = tree_legs(t, path_legs, nv, fixed_out, kept);
                std::vector<int> sl = sliced_legs ? user_sliced
                                                  : greedy_slice(t, legs, nv, forbidden, p.opts.max_log2_tensor,
                                                                 p.opts.n_sliced_target);
                std::vector<char> rem(fixed_out);
                for (int v : sl) rem[v] = 1;
                auto legs2 = tree_legs(t, path_legs, nv, rem, kept);
                double cost = tree_log2_cost_sum(t, legs2) + (double)sl.size();
                if (cost < best - 1e-9) {
                    best = cost;
                    p.tree = t;
                    p.sliced = sl;
                }
            }
        }
        // unsliced cost, for reporting
        {
            auto legs0 = tree_legs(p.tree, path_legs, nv, fixed_out, kept);
            p.info.flops_unsliced = 8.0 * std::exp2(tree_log2_cost_sum(p.tree, legs0));
        }
        if (p.sliced.size() > 62) fail(RQC_EPLAN, "more than 62 sliced legs");
        // -------- partial slicing (Alg. 1 and 2)
        const double f = p.opts.target_fidelity;
        const bool partial = f > 0 && f < 1;
        if (partial) fail(RQC_EINVAL, "partial slicing is not available in this build");
        // -------- batched legs: greedy, within the memory budget
        std::vector<int> cand;
        for (int v : p.sliced)
            if (std::find(p.S.begin(), p.S.end(), v) == p.S.end()) cand.push_back(v);
        std::vector<int> B;
        for (;;) {
            int bestv = -1;
            double best_key = 1e300;
            for (int v : cand) {
                if (std::find(B.begin(), B.end(), v) != B.end()) continue;
                std::vector<char> rem(fixed_out), kp(kept);
                for (int u : p.sliced) rem[u] = 1;
                for (int u : B) rem[u] = 0, kp[u] = 1;
                rem[v] = 0;
                kp[v] = 1;
                auto lg = tree_legs(p.tree, path_legs, nv, rem, kp);
                size_t mx = 0;
                double tot = 0;
                for (auto &l : lg) mx = std::max(mx, l.size()), tot += std::exp2((double)l.size());
                if ((int)mx > p.opts.max_log2_batched) continue;
                double key = (double)mx * 1e30 + tot;
                if (key < best_key) best_key = key, bestv = v;
            }
            if (bestv < 0) break;
            B.push_back(bestv);
        }
        // slice-id bit order: greedy-sliced legs are reordered batched-first so the
        // fixed FP64 summation order is ascending slice id; user legs keep their order
        if (!sliced_legs) {
            std::vector<int> ord;
            for (int v : p.sliced)
                if (std::find(B.begin(), B.end(), v) != B.end()) ord.push_back(v);
            for (int v : p.sliced)
                if (std::find(B.begin(), B.end(), v) == B.end()) ord.push_back(v);
            p.sliced = ord;
        }
        for (size_t t = 0; t < p.sliced.size(); t++) {
            int v = p.sliced[t];
            if (std::find(B.begin(), B.end(), v) != B.end()) {
                p.batched.push_back(v);
                p.batched_bit.push_back((int)t);
            } else {
                p.looped.push_back(v);
                p.looped_bit.push_back((int)t);
            }
        }
        // -------- final leg sets
        std::vector<char> rem(fixed_out), kp(kept);
        for (int v : p.looped) rem[v] = 1;
        for (int v : p.batched) kp[v] = 1;
        auto legs = tree_legs(p.tree, path_legs, nv, rem, kp);
        // projected variables
        std::vector<int> pidx(nv, -1);
        int np = 0;
        for (int q = 0; q < n; q++)
            if (!is_open[q]) {
                pidx[net.out_var[q]] = np++;
                p.fixed_qubit.push_back(q);
            }
        for (int v : p.looped) pidx[v] = np++;
        if (np > 256) fail(RQC_EPLAN, "more than 256 projected variables");
        // leaf buffer layout and selection descriptors
        p.n_leaves = (int)net.leaves.size();
        std::vector<int> leaf_off(p.n_leaves);
        std::vector<LeafSel> sel(p.n_leaves);
        int64_t full_off = 0, buf_off = 0;
        for (int i = 0; i < p.n_leaves; i++) {
            const Leaf &L = net.leaves[i];
            LeafSel d{};
            d.src = full_off;
            d.dst = buf_off;
            leaf_off[i] = (int)buf_off;
            for (size_t j = 0; j < L.legs.size(); j++) {
                int v = L.legs[j];
                if (std::binary_search(legs[i].begin(), legs[i].end(), v)) d.free_pos[d.n_free++] = (uint8_t)j;
                else if (pidx[v] >= 0) {
                    d.proj_pos[d.n_proj] = (uint8_t)j;
                    d.proj_idx[d.n_proj++] = (int16_t)pidx[v];
                } else
                    fail(RQC_EPLAN, "leaf leg neither kept nor projected");
            }
            sel[i] = d;
            full_off += (int64_t)L.data.size();
            buf_off += (int64_t)1 << legs[i].size();
        }
        // lower
        std::vector<int> root_layout;
        p.prog = lower_tree(p.tree, legs, leaf_off, root_layout);
        Program &pg = p.prog;
        pg.leafbuf_elems = buf_off;
        if ((size_t)pg.small_lds_elems * sizeof(float2) > 65536)
            fail(RQC_EPLAN, "fused subtree needs more than 64 KiB of LDS");
        {
            std::vector<int> om(n_open), sm(p.batched.size());
            for (int b = 0; b < n_open; b++) {
                int v = net.out_var[p.open_qubits[b]];
                auto it = std::find(root_layout.begin(), root_layout.end(), v);
                if (it == root_layout.end()) fail(RQC_EPLAN, "open leg missing from the final tensor");
                om[b] = (int)(it - root_layout.begin());
            }
            for (size_t u = 0; u < p.batched.size(); u++) {
                auto it = std::find(root_layout.begin(), root_layout.end(), p.batched[u]);
                if (it == root_layout.end()) fail(RQC_EPLAN, "batched leg missing from the final tensor");
                sm[u] = (int)(it - root_layout.begin());
            }
            if (root_layout.size() != (size_t)n_open + p.batched.size())
                fail(RQC_EPLAN, "final tensor has unexpected legs");
            pg.root_open = make_map(om);
            pg.root_slice = make_map(sm);
            pg.n_batched = (int)p.batched.size();
        }
        for (auto &op : pg.permutes) p.perm_desc.push_back(make_perm_desc(op.r, op.perm));
        // -------- device buffers
        std::vector<float2> full((size_t)full_off);
        {
            size_t k = 0;
            for (auto &L : net.leaves)
                for (auto &x : L.data) full[k++] = make_float2(x.real(), x.imag());
        }
        if (!p.opts.dry_run) try {
            p.d_full = (float2 *)p.dalloc(full.size() * sizeof(float2));
            p.d_sel = (LeafSel *)p.dalloc(sel.size() * sizeof(LeafSel));
            p.d_leafbuf = (float2 *)p.dalloc((size_t)buf_off * sizeof(float2));
            p.d_arena = (float2 *)p.dalloc((size_t)std::max<int64_t>(pg.arena_elems, 64) * sizeof(float2));
            p.d_steps = (SmallStep *)p.dalloc(std::max<size_t>(1, pg.small_steps.size()) * sizeof(SmallStep));
            p.d_trees = (SmallTree *)p.dalloc(std::max<size_t>(1, pg.small_trees.size()) * sizeof(SmallTree));
            p.d_acc = (double2 *)p.dalloc(((size_t)1 << n_open) * sizeof(double2));
            HIP_OK(hipMemcpy(p.d_full, full.data(), full.size() * sizeof(float2), hipMemcpyHostToDevice));
            HIP_OK(hipMemcpy(p.d_sel, sel.data(), sel.size() * sizeof(LeafSel), hipMemcpyHostToDevice));
            if (!pg.small_steps.empty())
                HIP_OK(hipMemcpy(p.d_steps, pg.small_steps.data(), pg.small_steps.size() * sizeof(SmallStep),
                                 hipMemcpyHostToDevice));
            if (!pg.small_trees.empty())
                HIP_OK(hipMemcpy(p.d_trees, pg.small_trees.data(), pg.small_trees.size() * sizeof(SmallTree),
                                 hipMemcpyHostToDevice));
        } catch (...) {
            p.release();
            throw;
        }
        // -------- info
        rqc_plan_info_t &I = p.info;
        I.n_qubits = n;
        I.n_open = n_open;
        I.n_variables = nv;
        I.n_sliced = (int32_t)p.sliced.size();
        I.n_batched = (int32_t)p.batched.size();
        I.n_partial = (int32_t)p.S.size();
        I.n_groups = (int64_t)1 << p.looped.size();
        I.n_slices = I.n_groups << p.batched.size();
        I.n_partial_kept = (int64_t)p.X.size();
        I.fidelity = p.F;
        I.flops_per_batch = pg.flops * (double)I.n_groups;
        I.gemm_flop_share = pg.flops > 0 ? pg.gemm_flops / pg.flops : 0.0;
        I.bytes_per_batch = pg.bytes * (double)I.n_groups;
        I.max_log2_tensor = pg.max_log2;
        I.n_steps = (int32_t)p.tree.steps.size();
        I.n_launches = (int32_t)pg.ops.size() + 2;
        I.workspace_bytes = 0;
        for (auto &o : p.owned) I.workspace_bytes += (int64_t)o.second;
        I.plan_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
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

rqc_status rqc_plan_partial(const rqc_plan *p, int32_t *S, int32_t capS, uint64_t *X, int64_t capX, double *R,
                            int64_t capR) {
    return guard([&] {
        if (!p) fail(RQC_EINVAL, "null plan");
        for (size_t i = 0; S && i < p->S.size() && (int64_t)i < capS; i++) S[i] = p->S[i];
        for (size_t i = 0; X && i < p->X.size() && (int64_t)i < capX; i++) X[i] = p->X[i];
        for (size_t i = 0; R && i < p->R.size() && (int64_t)i < capR; i++) R[i] = p->R[i];
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
    });
}

void rqc_plan_destroy(rqc_plan *p) {
    if (!p) return;
    if (!p->opts.dry_run) (void)hipDeviceSynchronize();
    p->release();
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
        hipStream_t s = (hipStream_t)hip_stream;
        const Program &pg = p->prog;
        // slice groups: values of the looped legs, ascending
        std::vector<uint64_t> groups;
        const int nl = (int)p->looped.size(), nb = (int)p->batched.size();
        if (!slice_ids) {
            for (uint64_t g = 0; g < ((uint64_t)1 << nl); g++) groups.push_back(g);
        } else {
            if (n_slices < 0) fail(RQC_EINVAL, "negative slice count");
            std::vector<std::pair<uint64_t, uint64_t>> kv; // (looped value, batched value)
            for (int64_t i = 0; i < n_slices; i++) {
                uint64_t sid = slice_ids[i];
                if (p->sliced.size() < 64 && (sid >> p->sliced.size()))
                    fail(RQC_EINVAL, "slice id has bits beyond the sliced legs");
                uint64_t lv = 0, bv = 0;
                for (int u = 0; u < nl; u++) lv |= ((sid >> p->looped_bit[u]) & 1) << u;
                for (int u = 0; u < nb; u++) bv |= ((sid >> p->batched_bit[u]) & 1) << u;
                kv.push_back({lv, bv});
            }
            std::sort(kv.begin(), kv.end());
            for (size_t i = 0; i < kv.size();) {
                size_t j = i;
                while (j < kv.size() && kv[j].first == kv[i].first) j++;
                if (j - i != ((size_t)1 << nb))
                    fail(RQC_EINVAL, "slice list must contain whole batched groups (" +
                                         std::to_string((size_t)1 << nb) + " slices per looped value)");
                for (size_t k = i; k < j; k++)
                    if (kv[k].second != (uint64_t)(k - i)) fail(RQC_EINVAL, "repeated slice id");
                groups.push_back(kv[i].first);
                i = j;
            }
        }
        const int n_open = (int)p->open_qubits.size();
        const int64_t nout = (int64_t)1 << n_open;
        const double scale = 1.0 / std::sqrt(p->F);
        const int nfix = (int)p->fixed_qubit.size();
        auto ptr = [&](const Buf &b) -> float2 * { return (b.kind == 0 ? p->d_arena : p->d_leafbuf) + b.off; };
        for (int64_t bi = 0; bi < n_batches; bi++) {
            {
                Timer t(p, s, RQC_K_ACCUM, 0, 16.0 * nout);
                launch_zero(p->d_acc, nout, s);
            }
            for (uint64_t g : groups) {
                ProjVals vals{};
                for (int i = 0; i < nfix; i++)
                    if ((fixed_bits[bi] >> p->fixed_qubit[i]) & 1) vals.w[i >> 6] |= 1ull << (i & 63);
                for (int u = 0; u < nl; u++)
                    if ((g >> u) & 1) {
                        int idx = nfix + u;
                        vals.w[idx >> 6] |= 1ull << (idx & 63);
                    }
                {
                    Timer t(p, s, RQC_K_LEAF, 0, 16.0 * (double)pg.leafbuf_elems);
                    launch_leaf_select(p->d_full, p->d_leafbuf, p->d_sel, p->n_leaves, vals, s);
                }
                for (const Op &op : pg.ops) {
                    switch (op.kind) {
                    case OP_SMALL: {
                        Timer t(p, s, RQC_K_SMALL, op.flops, op.bytes);
                        launch_small_trees(p->d_steps, p->d_trees, (int)pg.small_trees.size(), pg.small_lds_elems,
                                           p->d_leafbuf, p->d_arena, s);
                        break;
                    }
                    case OP_STREAM: {
                        const StreamOp &so = pg.streams[op.index];
                        Timer t(p, s, RQC_K_STREAM, op.flops, op.bytes);
                        launch_stream(so, ptr(so.a), ptr(so.b), ptr(so.c), s);
                        break;
                    }
                    case OP_PERMUTE: {
                        const PermuteOp &po = pg.permutes[op.index];
                        Timer t(p, s, RQC_K_PERMUTE, op.flops, op.bytes);
                        launch_permute(p->perm_desc[op.index], ptr(po.src), ptr(po.dst), s);
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
                        Timer t(p, s, RQC_K_GEMM, op.flops, op.bytes);
                        launch_gemm(ga, p->opts.precision, s);
                        break;
                    }
                    }
                }
                {
                    Timer t(p, s, RQC_K_ACCUM, 0, 8.0 * (double)(nout << nb) + 32.0 * nout);
                    launch_accumulate(ptr(pg.root), pg.root_open, pg.root_slice, n_open, nb, p->d_acc, s);
                }
            }
            {
                Timer t(p, s, RQC_K_FINAL, 0, 16.0 * nout + 8.0 * nout);
                launch_finalize(p->d_acc, nout, scale, (float2 *)out_amps + bi * nout,
                                out_f64 ? (double2 *)out_f64 + bi * nout : nullptr, s);
            }
        }
        HIP_OK(hipGetLastError());
        if (p->opts.profile && p->pending.size() > 8192) p->flush_profile();
    });
}

rqc_status rqc_rejection_sample(const void *amps, const uint64_t *fixed_bits, int64_t n_batches,
                                const int32_t *open_qubits, int32_t n_open, int32_t log2_NA, int32_t n_qubits,
                                double alpha, double F_norm, uint64_t seed, uint64_t batch_index_base,
                                int64_t pick_steps, int64_t n_samples, uint64_t *out_samples, int64_t *n_out,
                                rqc_sample_stats *stats, void *hip_stream) {
    rqc_status st = guard([&] {
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
        hipStream_t s = (hipStream_t)hip_stream;
        std::vector<uint64_t> fb(std::max<int64_t>(n_batches, 1), 0);
        for (int64_t i = 0; i < n_batches; i++) fb[i] = fixed_bits[i];
        std::vector<int32_t> oq(std::max(n_open, 1), 0);
        for (int b = 0; b < n_open; b++) oq[b] = open_qubits[b];
        uint64_t *d_fixed = nullptr;
        int32_t *d_open = nullptr;
        HIP_OK(hipMalloc(&d_fixed, fb.size() * sizeof(uint64_t)));
        hipError_t e = hipMalloc(&d_open, oq.size() * sizeof(int32_t));
        if (e != hipSuccess) {
            (void)hipFree(d_fixed);
            fail(RQC_EDEVICE, "hipMalloc failed");
        }
        e = hipMemcpyAsync(d_fixed, fb.data(), fb.size() * sizeof(uint64_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_open, oq.data(), oq.size() * sizeof(int32_t), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = run_sampler((const float2 *)amps, d_fixed, n_batches, d_open, n_open, log2_NA, n_qubits, alpha,
                            F_norm, seed, batch_index_base, pick_steps, n_samples, out_samples, n_out, stats, s);
        (void)hipStreamSynchronize(s);
        (void)hipFree(d_fixed);
        (void)hipFree(d_open);
        if (e != hipSuccess) fail(RQC_EDEVICE, std::string("sampler: ") + hipGetErrorString(e));
    });
    if (st == RQC_OK && *n_out < n_samples) {
        g_err = "fewer accepted samples than requested";
        return RQC_ESHORT;
    }
    return st;
}

} // extern "C"
