// Host planning: network specs, tree and slicing, partial-slice selection
// (Appendix B, Alg. 1 and 2) and the final lowering of a plan.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <thread>

#include "host.hpp"

namespace rqc {

Program lower_tree(const Tree &tree, const std::vector<Legs> &legs, const std::vector<int> &leaf_offsets,
                   const std::vector<char> &leaf_dep, bool cache, bool fuse, bool mx_streams,
                   std::vector<int> &root_layout);

void sort_leaf(Leaf &L) {
    std::vector<int> order(L.legs.size());
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int i, int j) { return L.legs[i] < L.legs[j]; });
    std::vector<int> nl(order.size());
    std::vector<cf> nd(L.data.size());
    for (size_t i = 0; i < order.size(); i++) nl[i] = L.legs[order[i]];
    for (size_t x = 0; x < nd.size(); x++) {
        size_t src = 0;
        for (size_t i = 0; i < order.size(); i++)
            if ((x >> i) & 1) src |= (size_t)1 << order[i];
        nd[x] = L.data[src];
    }
    L.legs = nl;
    L.data = nd;
}

NetSpec circuit_spec(const Network &net, const std::vector<int> &open_qubits) {
    NetSpec s;
    const int n = net.n_qubits;
    s.leaves = net.leaves;
    s.n_vars = net.n_vars;
    std::vector<char> is_open(n, 0);
    for (int q : open_qubits) {
        if (q < 0 || q >= n || is_open[q]) fail(RQC_EINVAL, "open qubits must be distinct and in range");
        is_open[q] = 1;
        s.open_vars.push_back(net.out_var[q]);
    }
    s.forbidden.assign(net.n_vars, 0);
    for (int v = 0; v < n; v++) s.forbidden[v] = 1;
    for (int q = 0; q < n; q++) {
        s.forbidden[net.out_var[q]] = 1;
        if (!is_open[q]) {
            s.fixed_vars.push_back(net.out_var[q]);
            s.fixed_bit.push_back(q);
        }
    }
    return s;
}

NetSpec doubled_spec(const Network &net, const std::vector<int> &S) {
    const int ng = (int)net.leaves.size(), nv = net.n_vars;
    std::vector<std::vector<int>> touch(nv);
    std::vector<int> created(ng, 0);
    for (int g = 0; g < ng; g++)
        for (int v : net.gate_inputs[g]) touch[v].push_back(g);
    for (int v = 0; v < nv; v++)
        if (net.var_gate[v] >= 0) created[net.var_gate[v]]++;
    // C_1: the causal past of the gates creating S
    std::vector<char> in1(ng, 0);
    std::vector<int> stack;
    for (int v : S) {
        if (v < 0 || v >= nv || net.var_gate[v] < 0) fail(RQC_EPLAN, "partially sliced vertex is not a gate output");
        stack.push_back(net.var_gate[v]);
    }
    while (!stack.empty()) {
        int g = stack.back();
        stack.pop_back();
        if (in1[g]) continue;
        in1[g] = 1;
        for (int v : net.gate_inputs[g]) {
            const auto &t = touch[v];
            int pos = (int)(std::find(t.begin(), t.end(), g) - t.begin());
            int pred = pos > 0 ? t[pos - 1] : net.var_gate[v];
            if (pred >= 0 && !in1[pred]) stack.push_back(pred);
        }
    }
    // variables consumed inside C_1 (input of a gate that creates new ones)
    std::vector<char> consumed(nv, 0);
    for (int g = 0; g < ng; g++)
        if (in1[g] && created[g] > 0)
            for (int v : net.gate_inputs[g]) consumed[v] = 1;
    for (int v : S)
        if (consumed[v]) fail(RQC_EPLAN, "partially sliced vertices are not an antichain");
    NetSpec s;
    s.n_vars = 2 * nv;
    for (int g = 0; g < ng; g++) {
        if (!in1[g]) continue;
        const Leaf &L = net.leaves[g];
        s.leaves.push_back(L);
        Leaf c = L;
        for (auto &x : c.data) x = std::conj(x);
        for (auto &v : c.legs)
            if (consumed[v]) v += nv;
        sort_leaf(c);
        s.leaves.push_back(c);
    }
    s.open_vars = S;
    s.forbidden.assign(s.n_vars, 0);
    for (int v : S) s.forbidden[v] = 1;
    return s;
}

static std::vector<Legs> leaf_leg_sets(const NetSpec &s, const std::vector<char> &drop) {
    std::vector<Legs> out;
    for (auto &L : s.leaves) {
        Legs l;
        for (int v : L.legs)
            if (!drop[v]) l.push_back(v);
        std::sort(l.begin(), l.end());
        out.push_back(l);
    }
    return out;
}

// Estimated GPU time of one batch under the plan from measured kernel rates:
// GEMM flops (8 per complex multiply-add) at the rate below, streaming and
// permute bytes at their measured HBM rates, a few microseconds per launch.
double estimate_seconds(const PlanCore &p) {
    const Program &pg = p.prog;
    // measured rates on MI355X, 8 flops per complex multiply-add: the complex64
    // GEMM takes three real products per multiply-add and runs at 129-170
    // TFLOP/s in this count (75-80 % of the FP32 MFMA peak executed), the split
    // GEMM at ~1/3 of its 3-product ceiling
    const double gemm_rate = p.opts.precision == RQC_C64 ? 1.0 * 157.3e12 : 0.33 * 838.9e12;
    // with the global cache a batch runs only the fixed-bit-dependent launches;
    // the rest is filled once and weighed as shared by many batches
    const double w_indep = pg.cache ? 1.0 / 256 : 1.0;
    double t = 20e-6;
    for (const Op &op : pg.ops) {
        double dt;
        // fixed cost per launch: the smallest streaming launches measure ~10 us
        // of kernel time on the 53-qubit plan, plus the gap to the next one
        if (op.kind == OP_GEMM) {
            dt = std::max(op.flops / gemm_rate, op.bytes / 5.5e12) + 8e-6;
        } else if (op.kind == OP_SMALL) {
            dt = 70e-6;
        } else if (op.kind == OP_PERMUTE) {
            dt = op.bytes / 5e12 + 8e-6;
        } else {
            // streaming kernels at their measured rates: matrix-core tiles
            // ~4.5 TB/s, long contractions ~2 TB/s plus their partial-sum pass,
            // the vector fallbacks under 1 TB/s
            const StreamOp &so = pg.streams[op.index];
            const double rate = so.mx || so.mx2 ? 4.5e12 : (so.lk ? 2e12 : 0.8e12);
            dt = op.bytes / rate + 10e-6;
            // a fused pair may be bound by its two matrix-core stages instead
            if (so.mx2) dt = std::max(dt, op.flops / (0.5 * 157.3e12) + 10e-6);
            if (so.lk && so.lk_split > 0) dt += 16.0 * std::exp2((double)(so.lk_split + so.nr + so.nf)) / 2e12 + 8e-6;
        }
        t += (op.kind == OP_SMALL || op.dep) ? dt : w_indep * dt;
    }
    return t * (double)std::max<int64_t>(1, p.info.n_groups);
}

int partial_k0(const rqc_plan_opts &o) {
    return o.partial_k > 0 ? o.partial_k : (int)std::ceil(3.0 - std::log2(o.target_fidelity));
}

// Simulated annealing of the best few searched results (tree, and sliced legs
// when slice_moves), one host thread each; the annealed results join the list,
// which is kept sorted by the proxy cost.
static void anneal_results(std::vector<SearchResult> &rs, const std::vector<Legs> &leaf_legs, int nv,
                           const std::vector<char> &kept, const std::vector<char> &forbidden,
                           const rqc_plan_opts &o, bool slice_moves, uint64_t seed) {
    if (o.anneal_iters <= 0 || rs.empty()) return;
    const int n = std::min<int>(4, (int)rs.size());
    std::vector<SearchResult> out(n);
    std::vector<std::thread> pool;
    for (int i = 0; i < n; i++)
        pool.emplace_back([&, i] {
            out[i] = anneal_tree(rs[i].tree, rs[i].sliced, leaf_legs, nv, kept, forbidden, o.max_log2_tensor,
                                 slice_moves, o.n_sliced_target, o.anneal_iters, seed * 0x9E3779B97F4A7C15ull + i);
        });
    for (auto &t : pool) t.join();
    for (auto &r : out) rs.push_back(std::move(r));
    std::stable_sort(rs.begin(), rs.end(),
                     [](const SearchResult &a, const SearchResult &b) { return a.log2cost < b.log2cost; });
}

void plan_tree(PlanCore &p, const int32_t *path, int32_t n_path_pairs, const std::vector<int> *user_sliced,
               const LightCones *lc) {
    const NetSpec &sp = p.spec;
    const int nv = sp.n_vars;
    std::vector<char> kept(nv, 0), fixed(nv, 0);
    for (int v : sp.open_vars) kept[v] = 1;
    for (int v : sp.fixed_vars) fixed[v] = 1;
    std::vector<Legs> path_legs = leaf_leg_sets(sp, fixed);
    p.user_legs = user_sliced != nullptr;
    if (user_sliced) {
        std::vector<char> seen(nv, 0);
        for (int v : *user_sliced) {
            if (v < 0 || v >= nv || sp.forbidden[v] || seen[v])
                fail(RQC_EINVAL, "sliced leg " + std::to_string(v) + " is not an internal variable");
            seen[v] = 1;
        }
    }
    if (path) {
        Tree t;
        t.n_leaves = (int)path_legs.size();
        std::vector<char> used(t.n_leaves + std::max(n_path_pairs, 0), 0);
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
        if (user_sliced) p.sliced = *user_sliced;
        else {
            auto legs = tree_legs(t, path_legs, nv, fixed, kept);
            p.sliced = greedy_slice(t, legs, nv, sp.forbidden, p.opts.max_log2_tensor, p.opts.n_sliced_target);
        }
    } else {
        int trials = p.opts.path_trials > 0 ? p.opts.path_trials : 16;
        std::vector<SearchResult> rs;
        if (lc && !user_sliced) {
            // partial slicing: S near the inputs first (Sec. I.B step 1), then
            // the tree for the network with S projected, then memory slicing
            std::vector<SearchResult> first = search_tree(path_legs, nv, kept, sp.forbidden, nullptr,
                                                          p.opts.max_log2_tensor, p.opts.n_sliced_target,
                                                          std::max(16, trials / 4), p.opts.path_seed);
            std::vector<char> none(nv, 0);
            // one candidate S from each of the best first trees (they differ in
            // which near-input legs carry the most cost); each gets its own
            // search, and all results compete below
            std::vector<std::vector<int>> tried;
            const int n_first = std::min<int>(4, (int)first.size());
            for (int fi = 0; fi < n_first; fi++) {
                auto legs_first = tree_legs(first[fi].tree, path_legs, nv, none, kept);
                // cones of at most 4 vertices: outputs of the first two
                // single-qubit layers in this gate set
                std::vector<int> S0 = near_input_select(first[fi].tree, legs_first, nv, sp.forbidden, *lc,
                                                        partial_k0(p.opts), 4);
                std::vector<int> key(S0);
                std::sort(key.begin(), key.end());
                if (std::find(tried.begin(), tried.end(), key) != tried.end()) continue;
                tried.push_back(key);
                std::vector<char> inS(nv, 0), forb(sp.forbidden);
                for (int v : S0) inS[v] = 1, forb[v] = 1;
                std::vector<Legs> reduced;
                for (auto &l : path_legs) {
                    Legs m;
                    for (int v : l)
                        if (!inS[v]) m.push_back(v);
                    reduced.push_back(m);
                }
                std::vector<SearchResult> part =
                    search_tree(reduced, nv, kept, forb, nullptr, p.opts.max_log2_tensor, p.opts.n_sliced_target,
                                std::max(16, trials / n_first), p.opts.path_seed + 1 + (uint64_t)fi);
                anneal_results(part, reduced, nv, kept, forb, p.opts, true, p.opts.path_seed + 1 + (uint64_t)fi);
                for (auto &r : part) {
                    r.sliced.insert(r.sliced.begin(), S0.begin(), S0.end());
                    r.log2cost += (double)S0.size();
                    rs.push_back(std::move(r));
                }
            }
            std::stable_sort(rs.begin(), rs.end(),
                             [](const SearchResult &a, const SearchResult &b) { return a.log2cost < b.log2cost; });
        } else if (user_sliced) {
            // the tree for the network with the given legs projected
            std::vector<char> inI(nv, 0);
            for (int v : *user_sliced) inI[v] = 1;
            std::vector<Legs> reduced;
            for (auto &l : path_legs) {
                Legs m;
                for (int v : l)
                    if (!inI[v]) m.push_back(v);
                reduced.push_back(m);
            }
            rs = search_tree(reduced, nv, kept, sp.forbidden, user_sliced, p.opts.max_log2_tensor,
                             p.opts.n_sliced_target, trials, p.opts.path_seed);
            anneal_results(rs, reduced, nv, kept, sp.forbidden, p.opts, false, p.opts.path_seed);
        } else {
            rs = search_tree(path_legs, nv, kept, sp.forbidden, nullptr, p.opts.max_log2_tensor,
                             p.opts.n_sliced_target, trials, p.opts.path_seed);
            anneal_results(rs, path_legs, nv, kept, sp.forbidden, p.opts, true, p.opts.path_seed);
        }
        // the best by the proxy cost are lowered and compared by estimated time
        // (with the global cache, the per-batch time the proxy does not see)
        const size_t n_lower = 64; // lowering a candidate costs ~10 ms
        p.candidates.clear();
        for (size_t i = 0; i < rs.size() && i < n_lower; i++) {
            PlanCore q;
            q.opts = p.opts;
            q.spec = p.spec;
            q.tree = rs[i].tree;
            q.sliced = rs[i].sliced;
            q.user_legs = p.user_legs;
            // a partial plan keeps its partially sliced legs looped: the
            // estimate must not batch them
            if (lc && !user_sliced) q.S = sliced_vertex_select(*lc, q.sliced, partial_k0(p.opts));
            try {
                plan_finish(q);
                p.candidates.push_back({rs[i].tree, rs[i].sliced, estimate_seconds(q)});
            } catch (const Error &) {
            }
        }
        if (p.candidates.empty()) fail(RQC_EPLAN, "no searched tree could be lowered");
        std::stable_sort(p.candidates.begin(), p.candidates.end(),
                         [](const PlanCore::Candidate &a, const PlanCore::Candidate &b) { return a.est < b.est; });
        p.tree = p.candidates[0].tree;
        p.sliced = p.candidates[0].sliced;
    }
    auto legs0 = tree_legs(p.tree, path_legs, nv, fixed, kept);
    p.info.flops_unsliced = 8.0 * std::exp2(tree_log2_cost_sum(p.tree, legs0));
    if (p.sliced.size() > 62) fail(RQC_EPLAN, "more than 62 sliced legs");
}

void plan_partial(PlanCore &p, const Network &net,
                  const std::function<std::vector<double>(const NetSpec &, const std::vector<int> &)> &norms) {
    const double f = p.opts.target_fidelity;
    const int k0 = partial_k0(p.opts);
    LightCones lc = light_cones(net);
    std::vector<int> S = sliced_vertex_select(lc, p.sliced, k0);
    if (S.empty()) fail(RQC_EPLAN, "no partially sliced vertex could be selected");
    if (S.size() > 30) fail(RQC_EPLAN, "more than 30 partially sliced vertices");
    std::vector<double> R = norms(doubled_spec(net, S), S);
    const size_t nR = (size_t)1 << S.size();
    if (R.size() != nR) fail(RQC_EPLAN, "norm tensor has the wrong size");
    std::vector<uint64_t> order(nR);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](uint64_t a, uint64_t b) { return R[a] > R[b]; });
    std::vector<uint64_t> X;
    double F = 0;
    if (p.opts.partial_total_slices > 0 || p.opts.partial_count > 0) {
        size_t cnt;
        if (p.opts.partial_total_slices > 0) {
            const double per = std::exp2((double)p.sliced.size() - (double)S.size());
            cnt = (size_t)std::max(1.0, std::floor((double)p.opts.partial_total_slices / per + 0.5));
        } else {
            cnt = (size_t)p.opts.partial_count;
        }
        cnt = std::min(cnt, nR);
        for (size_t i = 0; i < cnt; i++) X.push_back(order[i]), F += R[order[i]];
    } else {
        for (size_t i = 0; i < nR; i++) {
            X.push_back(order[i]);
            F += R[order[i]];
            if (F >= f) break;
        }
    }
    if (!(F > 0)) fail(RQC_EPLAN, "selected slices have zero norm");
    p.S = S;
    p.R = R;
    p.X = X;
    p.F = F;
}

void plan_finish(PlanCore &p) {
    const NetSpec &sp = p.spec;
    const int nv = sp.n_vars;
    std::vector<char> kept(nv, 0), fixed(nv, 0);
    for (int v : sp.open_vars) kept[v] = 1;
    for (int v : sp.fixed_vars) fixed[v] = 1;
    std::vector<Legs> path_legs = leaf_leg_sets(sp, fixed);
    auto in_S = [&](int v) { return std::find(p.S.begin(), p.S.end(), v) != p.S.end(); };
    // batched legs: greedy within the memory budget; partially sliced legs stay looped
    std::vector<int> B;
    for (;;) {
        int bestv = -1;
        double best_key = 1e300;
        for (int v : p.sliced) {
            if (in_S(v) || std::find(B.begin(), B.end(), v) != B.end()) continue;
            std::vector<char> rem(fixed), kp(kept);
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
    // slice-id bit order: searched legs go batched-first so the fixed FP64
    // summation order is ascending slice id; user-given legs keep their order
    if (!p.user_legs) {
        std::vector<int> ord;
        for (int v : p.sliced)
            if (std::find(B.begin(), B.end(), v) != B.end()) ord.push_back(v);
        for (int v : p.sliced)
            if (std::find(B.begin(), B.end(), v) == B.end()) ord.push_back(v);
        p.sliced = ord;
    }
    p.batched.clear();
    p.looped.clear();
    p.batched_bit.clear();
    p.looped_bit.clear();
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
    // default slice groups (values of the looped legs)
    p.groups.clear();
    p.n_group_range = 0;
    const int nl = (int)p.looped.size();
    if (p.S.empty() || p.X.empty()) {
        // no partial selection yet (a host-only plan): every slice, S looped
        if (nl > 62) fail(RQC_EPLAN, "too many looped slice legs");
        p.n_group_range = (uint64_t)1 << nl; // groups 0 .. 2^nl - 1, not materialised
    } else {
        if ((double)p.X.size() * std::exp2((double)(nl - (int)p.S.size())) > (double)(1 << 26))
            fail(RQC_EPLAN, "default partial slice list exceeds 2^26 groups");
        std::vector<int> s_pos(nl, -1); // looped leg -> index in S
        for (int u = 0; u < nl; u++)
            for (size_t t = 0; t < p.S.size(); t++)
                if (p.looped[u] == p.S[t]) s_pos[u] = (int)t;
        const int rest_bits = nl - (int)p.S.size();
        if (rest_bits > 40) fail(RQC_EPLAN, "too many looped slice legs for a default slice list");
        std::vector<uint64_t> xs(p.X);
        std::sort(xs.begin(), xs.end());
        for (uint64_t x : xs)
            for (uint64_t r = 0; r < ((uint64_t)1 << rest_bits); r++) {
                uint64_t g = 0;
                int rb = 0;
                for (int u = 0; u < nl; u++) {
                    uint64_t bit = s_pos[u] >= 0 ? (x >> s_pos[u]) & 1 : (r >> rb++) & 1;
                    g |= bit << u;
                }
                p.groups.push_back(g);
            }
    }
    // final leg sets
    std::vector<char> rem(fixed), kp(kept);
    for (int v : p.looped) rem[v] = 1;
    for (int v : p.batched) kp[v] = 1;
    auto legs = tree_legs(p.tree, path_legs, nv, rem, kp);
    // projected variables: fixed legs, then looped legs
    std::vector<int> pidx(nv, -1);
    int np = 0;
    for (int v : sp.fixed_vars) pidx[v] = np++;
    for (int v : p.looped) pidx[v] = np++;
    if (np > 256) fail(RQC_EPLAN, "more than 256 projected variables");
    const int nleaves = (int)sp.leaves.size();
    std::vector<int> leaf_off(nleaves);
    p.sel.assign(nleaves, LeafSel{});
    int64_t full_off = 0, buf_off = 0;
    for (int i = 0; i < nleaves; i++) {
        const Leaf &L = sp.leaves[i];
        if (L.legs.size() > 4) fail(RQC_EPLAN, "leaf with more than 4 legs");
        LeafSel d{};
        d.src = full_off;
        buf_off = (buf_off + 1) & ~(int64_t)1; // 16-byte aligned tensors
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
        p.sel[i] = d;
        full_off += (int64_t)L.data.size();
        buf_off += (int64_t)1 << legs[i].size();
    }
    p.full.clear();
    p.full.reserve((size_t)full_off);
    double log2_kappa = 0;
    for (auto &L : sp.leaves) {
        p.full.insert(p.full.end(), L.data.begin(), L.data.end());
        log2_kappa -= std::log2(L.scale);
    }
    p.kappa = std::exp2(log2_kappa);
    if (!(p.kappa > 0) || !std::isfinite(p.kappa)) fail(RQC_EPLAN, "leaf scale product out of range");
    std::vector<int> root_layout;
    // leaves that carry a fixed output bit; everything below them depends on
    // the batch, the rest only on the slice group
    std::vector<char> is_fixed(sp.n_vars, 0), leaf_dep(nleaves, 0);
    for (int v : sp.fixed_vars) is_fixed[v] = 1;
    for (int i = 0; i < nleaves; i++)
        for (int v : sp.leaves[i].legs)
            if (is_fixed[v]) leaf_dep[i] = 1;
    p.prog = lower_tree(p.tree, legs, leaf_off, leaf_dep, p.opts.global_cache != 0, p.opts.no_stream_fusion == 0,
                        p.opts.no_matrix_core_streams == 0, root_layout);
    Program &pg = p.prog;
    pg.leafbuf_elems = buf_off;
    if ((size_t)pg.small_lds_elems * 8 > 65536) fail(RQC_EPLAN, "fused subtree needs more than 64 KiB of LDS");
    const int n_open = (int)sp.open_vars.size();
    std::vector<int> om(n_open), sm(p.batched.size());
    for (int b = 0; b < n_open; b++) {
        auto it = std::find(root_layout.begin(), root_layout.end(), sp.open_vars[b]);
        if (it == root_layout.end()) fail(RQC_EPLAN, "open leg missing from the final tensor");
        om[b] = (int)(it - root_layout.begin());
    }
    for (size_t u = 0; u < p.batched.size(); u++) {
        auto it = std::find(root_layout.begin(), root_layout.end(), p.batched[u]);
        if (it == root_layout.end()) fail(RQC_EPLAN, "batched leg missing from the final tensor");
        sm[u] = (int)(it - root_layout.begin());
    }
    if (root_layout.size() != (size_t)n_open + p.batched.size()) fail(RQC_EPLAN, "final tensor has unexpected legs");
    pg.root_open = make_map(om);
    pg.root_slice = make_map(sm);
    pg.n_batched = (int)p.batched.size();
    rqc_plan_info_t &I = p.info;
    I.n_open = n_open;
    I.n_variables = nv;
    I.n_sliced = (int32_t)p.sliced.size();
    I.n_batched = (int32_t)p.batched.size();
    I.n_partial = (int32_t)p.S.size();
    I.n_groups = p.n_group_range ? (int64_t)p.n_group_range : (int64_t)p.groups.size();
    I.n_slices = I.n_groups << p.batched.size();
    I.n_partial_kept = (int64_t)p.X.size();
    I.fidelity = p.F;
    I.flops_per_batch = pg.flops * (double)I.n_groups;
    I.gemm_flop_share = pg.flops > 0 ? pg.gemm_flops / pg.flops : 0.0;
    I.bytes_per_batch = pg.bytes * (double)I.n_groups;
    I.max_log2_tensor = pg.max_log2;
    I.n_steps = (int32_t)p.tree.steps.size();
    I.n_launches = (int32_t)pg.ops.size() + 2;
    if (pg.cache) {
        // one cache block per slice group of the default list, plus one for
        // calls with their own slice list (recomputed there on every call)
        const double bytes = 8.0 * (double)pg.cache_elems * (double)(I.n_groups + 1);
        if (bytes > 128.0 * (1ull << 30))
            fail(RQC_EPLAN, "global cache would need " + std::to_string(bytes / (1ull << 30)) + " GiB");
        I.cache_bytes = (int64_t)bytes;
        I.flops_cached = pg.flops_indep * (double)I.n_groups;
    }
    I.est_seconds = estimate_seconds(p);
    I.n_fused = 0;
    for (int k = 0; k < SK_COUNT; k++) I.stream_kernels[k] = 0;
    for (const StreamOp &so : pg.streams) {
        I.n_fused += so.mx2;
        I.stream_kernels[stream_kernel(so)]++;
    }
}

// One line per op of the launch program: kind, kernel, shape, work.
std::string describe_program(const PlanCore &p) {
    static const char *sk_name[SK_COUNT] = {"mx2", "mx", "lk", "ky", "tile", "gen"};
    const Program &pg = p.prog;
    std::string out;
    char line[512];
    std::snprintf(line, sizeof line, "# op kind kernel dep flops bytes shape\n");
    out += line;
    for (size_t i = 0; i < pg.ops.size(); i++) {
        const Op &op = pg.ops[i];
        std::string shape;
        const char *kind = "?", *kern = "-";
        switch (op.kind) {
        case OP_SMALL:
            kind = "small";
            kern = "small_trees";
            std::snprintf(line, sizeof line, "trees=%zu lds_elems=%d", pg.small_trees.size(), pg.small_lds_elems);
            shape = line;
            break;
        case OP_STREAM: {
            const StreamOp &so = pg.streams[op.index];
            kind = "stream";
            kern = so.mx && so.wide ? "mx-wide" : sk_name[stream_kernel(so)];
            std::snprintf(line, sizeof line, "rc=%d nr=%d kc=%d nf=%d tile_l=%d lk_split=%d kc2=%d nf2=%d", so.rc, so.nr,
                          so.kc, so.nf, so.tile_l, so.lk_split, so.kc2, so.nf2);
            shape = line;
            break;
        }
        case OP_PERMUTE: {
            const PermuteOp &po = pg.permutes[op.index];
            kind = "permute";
            kern = "permute";
            std::snprintf(line, sizeof line, "r=%d", po.r);
            shape = line;
            break;
        }
        case OP_GEMM: {
            const GemmOp &go = pg.gemms[op.index];
            kind = "gemm";
            kern = "cgemm";
            std::snprintf(line, sizeof line, "batch=%lld M=%lld N=%lld K=%lld a_kfast=%d b_nfast=%d ksplit=%d",
                          (long long)go.batch, (long long)go.M, (long long)go.N, (long long)go.K, go.a_kfast, go.b_nfast,
                          go.ksplit);
            shape = line;
            if (go.c_ins_bits > 0) shape += " c_ins=" + std::to_string(go.c_ins_pos) + "/" + std::to_string(go.c_ins_bits);
            break;
        }
        }
        std::snprintf(line, sizeof line, "%zu %s %s %d %.6g %.6g ", i, kind, kern, op.dep, op.flops, op.bytes);
        out += line;
        out += shape;
        out += "\n";
    }
    return out;
}

} // namespace rqc
