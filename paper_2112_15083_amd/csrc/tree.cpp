// Contraction tree search (randomised greedy), leg bookkeeping and the
// greedy slicer.
//
// The contraction tree T and the sliced variables I are the inputs of the
// paper's method (Sec. I and Sec. I.B); the paper optimises them by simulated
// annealing in its simulator.  Here: a greedy pairwise order that minimises
// |C| - |A| - |B| per step, randomised over several trials, then slicing legs
// one at a time, each chosen to minimise the total sliced cost among the legs
// of the largest tensors (or among all legs once the memory target holds).
#include <algorithm>
#include <numeric>
#include <atomic>
#include <functional>
#include <thread>
#include <cmath>
#include <queue>
#include <random>
#include <unordered_map>

#include "host.hpp"

namespace rqc {

static Legs merge_union(const Legs &a, const Legs &b) {
    Legs out;
    out.reserve(a.size() + b.size());
    std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(out));
    return out;
}

std::vector<Legs> tree_legs(const Tree &t, const std::vector<Legs> &leaf_legs, int n_vars,
                            const std::vector<char> &removed, const std::vector<char> &kept) {
    // total occurrence count of each variable over the leaves
    std::vector<int> total(n_vars, 0);
    for (auto &L : leaf_legs)
        for (int v : L)
            if (!removed[v]) total[v]++;
    const int nt = t.n_leaves + (int)t.steps.size();
    std::vector<Legs> legs(nt);
    // per tensor: occurrence counts of its own legs within its subtree
    std::vector<std::vector<int>> cnt(nt);
    for (int i = 0; i < t.n_leaves; i++) {
        for (int v : leaf_legs[i])
            if (!removed[v]) {
                legs[i].push_back(v);
                cnt[i].push_back(1);
            }
    }
    for (size_t s = 0; s < t.steps.size(); s++) {
        int a = t.steps[s].first, b = t.steps[s].second, c = t.n_leaves + (int)s;
        const Legs &A = legs[a], &B = legs[b];
        size_t i = 0, j = 0;
        Legs out;
        std::vector<int> oc;
        while (i < A.size() || j < B.size()) {
            int v;
            int k = 0;
            if (j >= B.size() || (i < A.size() && A[i] < B[j])) {
                v = A[i];
                k = cnt[a][i++];
            } else if (i >= A.size() || B[j] < A[i]) {
                v = B[j];
                k = cnt[b][j++];
            } else {
                v = A[i];
                k = cnt[a][i++] + cnt[b][j++];
            }
            if (kept[v] || k < total[v]) {
                out.push_back(v);
                oc.push_back(k);
            }
        }
        legs[c] = std::move(out);
        cnt[c] = std::move(oc);
        // operands are consumed: free their counts
        std::vector<int>().swap(cnt[a]);
        std::vector<int>().swap(cnt[b]);
    }
    return legs;
}

double tree_log2_cost_sum(const Tree &t, const std::vector<Legs> &legs) {
    // log2 of sum over steps of 2^|A u B|, computed stably
    double mx = -1;
    std::vector<int> r(t.steps.size());
    for (size_t s = 0; s < t.steps.size(); s++) {
        Legs u = merge_union(legs[t.steps[s].first], legs[t.steps[s].second]);
        r[s] = (int)u.size();
        mx = std::max(mx, (double)r[s]);
    }
    if (t.steps.empty()) return 0;
    double acc = 0;
    for (int x : r) acc += std::exp2((double)x - mx);
    return mx + std::log2(acc);
}

// Time-like cost of one pairwise step: complex multiply-adds plus kTraffic per
// element read or written.  On MI355X one complex64 element of HBM traffic
// (8 bytes at 8 TB/s) takes as long as ~20 complex MACs on FP32 MFMA
// (8 flops each at 157 TFLOP/s); a lower weight is used because small
// operands are served from cache or LDS.
static constexpr double kTraffic = 5.0;
// With `launches`: a step with a tensor above 2^10 elements is a kernel
// launch of its own (the smaller ones run fused in one launch of whole
// subtrees), and a launch takes ~8 us however little it does, the time of
// ~2^27 complex MACs on the matrix cores.  The greedy search scores without
// it; the annealer, whose moves can split work into many small steps, with it.
static constexpr double kLaunch = 134217728.0;
static constexpr int kFusedMaxRank = 10;

double step_time_cost(int ra, int rb, int runion, int rc, bool launches) {
    const double launch = launches && std::max(ra, std::max(rb, rc)) > kFusedMaxRank ? kLaunch : 0.0;
    return std::exp2((double)runion) +
           kTraffic * (std::exp2((double)ra) + std::exp2((double)rb) + std::exp2((double)rc)) + launch;
}

double tree_log2_time_cost(const Tree &t, const std::vector<Legs> &legs) {
    double acc = 0;
    for (size_t s = 0; s < t.steps.size(); s++) {
        const Legs &A = legs[t.steps[s].first], &B = legs[t.steps[s].second];
        Legs u = merge_union(A, B);
        acc += step_time_cost((int)A.size(), (int)B.size(), (int)u.size(),
                         (int)legs[t.n_leaves + s].size());
    }
    return std::log2(std::max(acc, 1.0));
}

namespace {
struct Cand {
    double key;
    int a, b;
    bool operator<(const Cand &o) const { return key > o.key; } // min-heap
};
} // namespace

Tree greedy_tree(const std::vector<Legs> &leaf_legs, int n_vars, const std::vector<char> &kept,
                 uint64_t seed, double temperature, double costmod) {
    const int n0 = (int)leaf_legs.size();
    std::vector<Legs> legs(leaf_legs);
    legs.reserve(2 * n0);
    std::vector<char> alive(n0, 1);
    std::vector<int> count(n_vars, 0);
    std::vector<std::vector<int>> holders(n_vars);
    for (int i = 0; i < n0; i++)
        for (int v : legs[i]) {
            count[v]++;
            holders[v].push_back(i);
        }
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> U(1e-12, 1.0);

    auto out_legs = [&](int a, int b) {
        const Legs &A = legs[a], &B = legs[b];
        Legs out;
        size_t i = 0, j = 0;
        while (i < A.size() || j < B.size()) {
            int v, k;
            if (j >= B.size() || (i < A.size() && A[i] < B[j])) {
                v = A[i++];
                k = 1;
            } else if (i >= A.size() || B[j] < A[i]) {
                v = B[j++];
                k = 1;
            } else {
                v = A[i++];
                j++;
                k = 2;
            }
            if (kept[v] || count[v] > k) out.push_back(v);
        }
        return out;
    };
    auto score = [&](int a, int b) {
        double sc = std::exp2((double)out_legs(a, b).size()) -
                    costmod * (std::exp2((double)legs[a].size()) + std::exp2((double)legs[b].size()));
        double key = (sc >= 0 ? 1 : -1) * std::log2(1.0 + std::fabs(sc));
        if (temperature > 0) key -= temperature * (-std::log(-std::log(U(rng))));
        return key;
    };

    std::priority_queue<Cand> heap;
    auto push_neighbours = [&](int t) {
        std::vector<int> nb;
        for (int v : legs[t])
            for (int u : holders[v])
                if (u != t && alive[u]) nb.push_back(u);
        std::sort(nb.begin(), nb.end());
        nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
        for (int u : nb) heap.push({score(std::min(t, u), std::max(t, u)), std::min(t, u), std::max(t, u)});
    };
    for (int i = 0; i < n0; i++) {
        std::vector<int> nb;
        for (int v : legs[i])
            for (int u : holders[v])
                if (u > i) nb.push_back(u);
        std::sort(nb.begin(), nb.end());
        nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
        for (int u : nb) heap.push({score(i, u), i, u});
    }
    Tree tree;
    tree.n_leaves = n0;
    auto merge = [&](int a, int b) {
        Legs C = out_legs(a, b);
        int t = (int)legs.size();
        for (int v : legs[a]) count[v]--;
        for (int v : legs[b]) count[v]--;
        for (int v : C) {
            count[v]++;
            holders[v].push_back(t);
        }
        legs.push_back(C);
        alive[a] = alive[b] = 0;
        alive.push_back(1);
        tree.steps.push_back({a, b});
        return t;
    };
    while (!heap.empty()) {
        Cand c = heap.top();
        heap.pop();
        if (!alive[c.a] || !alive[c.b]) continue;
        // counts may have changed since the candidate was scored: rescore once
        double now = score(c.a, c.b);
        if (now > c.key + 1e-9 && !heap.empty() && now > heap.top().key) {
            heap.push({now, c.a, c.b});
            continue;
        }
        int t = merge(c.a, c.b);
        push_neighbours(t);
    }
    // disconnected remainder: outer products, smallest first
    std::vector<int> rest;
    for (int i = 0; i < (int)alive.size(); i++)
        if (alive[i]) rest.push_back(i);
    while (rest.size() > 1) {
        std::sort(rest.begin(), rest.end(), [&](int x, int y) {
            return legs[x].size() != legs[y].size() ? legs[x].size() > legs[y].size() : x > y;
        });
        int a = rest.back();
        rest.pop_back();
        int b = rest.back();
        rest.pop_back();
        rest.push_back(merge(std::min(a, b), std::max(a, b)));
    }
    return tree;
}

// ------------------------------------------------------------------ subtree reconfiguration
namespace {
constexpr int kWords = 8; // local leg universe of up to 512 legs
struct Mask {
    uint64_t w[kWords];
};
inline Mask mor(const Mask &a, const Mask &b) {
    Mask r;
    for (int i = 0; i < kWords; i++) r.w[i] = a.w[i] | b.w[i];
    return r;
}
inline Mask mand(const Mask &a, const Mask &b) {
    Mask r;
    for (int i = 0; i < kWords; i++) r.w[i] = a.w[i] & b.w[i];
    return r;
}
inline int mpop(const Mask &a) {
    int c = 0;
    for (int i = 0; i < kWords; i++) c += __builtin_popcountll(a.w[i]);
    return c;
}
} // namespace

Tree reconfigure_tree(const Tree &t, const std::vector<Legs> &leaf_legs, int n_vars, const std::vector<char> &kept,
                      int k, int passes) {
    const int L = t.n_leaves, ns = (int)t.steps.size();
    if (ns < 2 || k < 3) return t;
    const int nt = L + ns;
    std::vector<int> ca(nt, -1), cb(nt, -1);
    for (int s = 0; s < ns; s++) ca[L + s] = t.steps[s].first, cb[L + s] = t.steps[s].second;
    const int root = nt - 1;
    std::vector<int> total(n_vars, 0);
    for (auto &l : leaf_legs)
        for (int v : l) total[v]++;
    std::vector<Legs> legs(nt);
    std::vector<std::vector<int>> cnt(nt);
    // post-order list of internal nodes
    auto postorder = [&]() {
        std::vector<int> order, stack{root};
        std::vector<char> done(nt, 0);
        while (!stack.empty()) {
            int u = stack.back();
            if (u < L) {
                stack.pop_back();
                continue;
            }
            if (!done[u]) {
                done[u] = 1;
                stack.push_back(ca[u]);
                stack.push_back(cb[u]);
            } else {
                stack.pop_back();
                order.push_back(u);
            }
        }
        return order;
    };
    auto compute_legs = [&](const std::vector<int> &order) {
        for (int i = 0; i < L; i++) {
            legs[i] = leaf_legs[i];
            cnt[i].assign(legs[i].size(), 1);
        }
        for (int c : order) {
            int a = ca[c], b = cb[c];
            const Legs &A = legs[a], &B = legs[b];
            Legs out;
            std::vector<int> oc;
            size_t i = 0, j = 0;
            while (i < A.size() || j < B.size()) {
                int v, kk;
                if (j >= B.size() || (i < A.size() && A[i] < B[j])) v = A[i], kk = cnt[a][i++];
                else if (i >= A.size() || B[j] < A[i]) v = B[j], kk = cnt[b][j++];
                else v = A[i], kk = cnt[a][i++] + cnt[b][j++];
                if (kept[v] || kk < total[v]) out.push_back(v), oc.push_back(kk);
            }
            legs[c] = out;
            cnt[c] = oc;
        }
    };
    for (int pass = 0; pass < passes; pass++) {
        std::vector<int> order = postorder();
        compute_legs(order);
        bool changed = false;
        for (int tnode : order) {
            // frontier: expand the largest internal members until k tensors
            std::vector<int> front{ca[tnode], cb[tnode]};
            std::vector<int> inner{tnode};
            while ((int)front.size() < k) {
                int best = -1;
                for (int i = 0; i < (int)front.size(); i++)
                    if (front[i] >= L && (best < 0 || legs[front[i]].size() > legs[front[best]].size())) best = i;
                if (best < 0) break;
                int u = front[best];
                inner.push_back(u);
                front[best] = ca[u];
                front.push_back(cb[u]);
            }
            const int f = (int)front.size();
            if (f < 3) continue;
            // local leg universe
            std::vector<int> uni;
            for (int u : front) uni.insert(uni.end(), legs[u].begin(), legs[u].end());
            std::sort(uni.begin(), uni.end());
            uni.erase(std::unique(uni.begin(), uni.end()), uni.end());
            if ((int)uni.size() > 64 * kWords) continue;
            auto to_mask = [&](const Legs &l) {
                Mask m{};
                for (int v : l) {
                    int i = (int)(std::lower_bound(uni.begin(), uni.end(), v) - uni.begin());
                    if (i < (int)uni.size() && uni[i] == v) m.w[i >> 6] |= 1ull << (i & 63);
                }
                return m;
            };
            std::vector<Mask> fm(f);
            for (int i = 0; i < f; i++) fm[i] = to_mask(legs[front[i]]);
            const Mask outside = to_mask(legs[tnode]);
            const int full = (1 << f) - 1;
            std::vector<Mask> U(1 << f);
            U[0] = Mask{};
            for (int S = 1; S <= full; S++) {
                int low = __builtin_ctz(S);
                U[S] = mor(U[S & (S - 1)], fm[low]);
            }
            std::vector<Mask> LG(1 << f);
            std::vector<int> lsz(1 << f);
            for (int S = 1; S <= full; S++) {
                LG[S] = mand(U[S], mor(outside, U[full ^ S]));
                lsz[S] = mpop(LG[S]);
            }
            std::vector<double> cost(1 << f, 0.0);
            std::vector<int> split(1 << f, 0);
            for (int S = 1; S <= full; S++) {
                if ((S & (S - 1)) == 0) continue;
                int low = S & -S, rest = S ^ low;
                double best = 1e300;
                int bs = 0;
                for (int sub = rest;; sub = (sub - 1) & rest) {
                    int S1 = low | sub, S2 = S ^ S1;
                    if (S2) {
                        double c = cost[S1] + cost[S2] +
                                   step_time_cost(lsz[S1], lsz[S2], mpop(mor(LG[S1], LG[S2])), lsz[S]);
                        if (c < best) best = c, bs = S1;
                    }
                    if (sub == 0) break;
                }
                cost[S] = best;
                split[S] = bs;
            }
            // old cost of the same subtree
            double old = 0;
            for (int u : inner)
                old += step_time_cost((int)legs[ca[u]].size(), (int)legs[cb[u]].size(),
                                 (int)merge_union(legs[ca[u]], legs[cb[u]]).size(), (int)legs[u].size());
            if (cost[full] >= old * (1 - 1e-9)) continue;
            // rebuild: reuse the inner node ids, tnode stays the subtree root
            std::vector<int> ids(inner.begin() + 1, inner.end());
            std::function<int(int, bool)> build = [&](int S, bool top) -> int {
                if ((S & (S - 1)) == 0) return front[__builtin_ctz(S)];
                int id;
                if (top) id = tnode;
                else {
                    id = ids.back();
                    ids.pop_back();
                }
                int S1 = split[S];
                int a = build(S1, false), b = build(S ^ S1, false);
                ca[id] = a;
                cb[id] = b;
                Legs l;
                for (int i = 0; i < (int)uni.size(); i++)
                    if ((LG[S].w[i >> 6] >> (i & 63)) & 1) l.push_back(uni[i]);
                legs[id] = l;
                return id;
            };
            build(full, true);
            changed = true;
            // counts of the rebuilt nodes are refreshed at the next pass
        }
        if (!changed) break;
    }
    // back to SSA order
    std::vector<int> order = postorder();
    std::vector<int> newid(nt, -1);
    for (int i = 0; i < L; i++) newid[i] = i;
    Tree out;
    out.n_leaves = L;
    for (int c : order) {
        out.steps.push_back({newid[ca[c]], newid[cb[c]]});
        newid[c] = L + (int)out.steps.size() - 1;
    }
    return out;
}

// Two phases: `trials` randomised greedy trees are built and scored by the
// time-like cost of the unsliced tree (cheap); the best sixteenth of them (at
// least 8) are rebuilt from their seeds, re-optimised by subtree
// reconfiguration (the expensive part) and sliced, and scored again.
std::vector<SearchResult> search_tree(const std::vector<Legs> &leaf_legs, int n_vars, const std::vector<char> &kept,
                                      const std::vector<char> &forbidden, const std::vector<int> *user_sliced,
                                      int max_log2_tensor, int n_target, int trials, uint64_t seed) {
    std::vector<char> none(n_vars, 0);
    auto greedy = [&](int tr) {
        std::mt19937_64 rng(seed * 0x9E3779B97F4A7C15ull + (uint64_t)tr);
        std::uniform_real_distribution<double> U(0.0, 1.0);
        double temp = tr == 0 ? 0.0 : 0.05 + 0.95 * U(rng);
        double costmod = tr == 0 ? 1.0 : 0.5 + 1.5 * U(rng);
        return greedy_tree(leaf_legs, n_vars, kept, rng(), temp, costmod);
    };
    const int nth = (int)std::max(1u, std::min<unsigned>(16u, std::thread::hardware_concurrency()));
    auto parallel = [&](int n, const std::function<void(int)> &fn) {
        std::atomic<int> next{0};
        std::vector<std::thread> pool;
        for (int i = 0; i < std::min(nth, n); i++)
            pool.emplace_back([&] {
                for (int k = next++; k < n; k = next++) fn(k);
            });
        for (auto &th : pool) th.join();
    };
    std::vector<double> score(trials);
    parallel(trials, [&](int tr) {
        Tree t = greedy(tr);
        score[tr] = tree_log2_time_cost(t, tree_legs(t, leaf_legs, n_vars, none, kept));
    });
    std::vector<int> order(trials);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return score[x] < score[y]; });
    const int keep = std::min(trials, std::max(8, trials / 16));
    std::vector<SearchResult> res(keep);
    parallel(keep, [&](int i) {
        Tree t = reconfigure_tree(greedy(order[i]), leaf_legs, n_vars, kept, 8, 3);
        auto legs = tree_legs(t, leaf_legs, n_vars, none, kept);
        std::vector<int> sl =
            user_sliced ? *user_sliced : greedy_slice(t, legs, n_vars, forbidden, max_log2_tensor, n_target);
        std::vector<char> rem(n_vars, 0);
        for (int v : sl) rem[v] = 1;
        auto legs2 = tree_legs(t, leaf_legs, n_vars, rem, kept);
        res[i] = {t, sl, tree_log2_time_cost(t, legs2) + (double)sl.size()};
    });
    std::stable_sort(res.begin(), res.end(),
                     [](const SearchResult &a, const SearchResult &b) { return a.log2cost < b.log2cost; });
    return res;
}

std::vector<int> greedy_slice(const Tree &t, const std::vector<Legs> &legs, int n_vars,
                              const std::vector<char> &forbidden, int max_log2_tensor, int n_target) {
    std::vector<char> sl(n_vars, 0);
    std::vector<int> out;
    const int nt = (int)legs.size();
    const int ns = (int)t.steps.size();
    std::vector<Legs> unions(ns);
    for (int s = 0; s < ns; s++) unions[s] = merge_union(legs[t.steps[s].first], legs[t.steps[s].second]);
    for (;;) {
        // sizes after current slicing
        int maxr = 0;
        for (int i = 0; i < nt; i++) {
            int r = 0;
            for (int v : legs[i]) r += !sl[v];
            maxr = std::max(maxr, r);
        }
        bool mem_ok = max_log2_tensor <= 0 || maxr <= max_log2_tensor;
        bool cnt_ok = n_target < 0 || (int)out.size() >= n_target;
        if (mem_ok && cnt_ok) break;
        // weight[v] = sum over steps containing v of the step's current cost
        std::vector<double> w(n_vars, 0.0);
        double mxr = 0;
        std::vector<int> rs(ns);
        for (int s = 0; s < ns; s++) {
            int r = 0;
            for (int v : unions[s]) r += !sl[v];
            rs[s] = r;
            mxr = std::max(mxr, (double)r);
        }
        for (int s = 0; s < ns; s++) {
            double c = std::exp2((double)rs[s] - mxr);
            for (int v : unions[s])
                if (!sl[v]) w[v] += c;
        }
        std::vector<char> cand(n_vars, 0);
        bool any = false;
        if (!mem_ok) {
            for (int i = 0; i < nt; i++) {
                int r = 0;
                for (int v : legs[i]) r += !sl[v];
                if (r == maxr)
                    for (int v : legs[i])
                        if (!sl[v] && !forbidden[v]) cand[v] = 1, any = true;
            }
        } else {
            for (int s = 0; s < ns; s++)
                for (int v : unions[s])
                    if (!sl[v] && !forbidden[v]) cand[v] = 1, any = true;
        }
        if (!any) break;
        int best = -1;
        for (int v = 0; v < n_vars; v++)
            if (cand[v] && (best < 0 || w[v] > w[best] * (1 + 1e-12))) best = v;
        sl[best] = 1;
        out.push_back(best);
    }
    return out;
}

// ------------------------------------------------------------------ light cones
LightCones light_cones(const Network &net) {
    // gates in the causal past of each gate (inclusive), as sorted lists of
    // input variables; computed with per-qubit cone sets over gate lines.
    const int n = net.n_qubits;
    const int ng = (int)net.leaves.size();
    // qubit of each current variable, to follow wires
    LightCones lc;
    lc.cone_vertices.assign(net.n_vars, {});
    // cone of a gate = union of cones of its input variables' creators + its own inputs
    std::vector<std::vector<int>> gate_cone(ng); // sorted vertex lists
    // the gate that last touched each variable's wire: for a variable v, the gates
    // that act on it (its creator, diagonal gates on it, its consumer) are ordered;
    // the causal past of gate g is the union of the past of the latest earlier gate
    // on each of g's input wires.
    std::vector<int> last_gate_on_var(net.n_vars, -1);
    for (int g = 0; g < ng; g++) {
        Legs acc;
        for (int v : net.gate_inputs[g]) {
            int h = last_gate_on_var[v] >= 0 ? last_gate_on_var[v] : net.var_gate[v];
            if (h >= 0) acc = merge_union(acc, gate_cone[h]);
        }
        Legs own(net.gate_inputs[g]);
        std::sort(own.begin(), own.end());
        gate_cone[g] = merge_union(acc, own);
        for (int v : net.gate_inputs[g]) last_gate_on_var[v] = g;
        // outputs of this gate start their wire history here
        (void)n;
    }
    for (int v = 0; v < net.n_vars; v++)
        if (net.var_gate[v] >= 0) lc.cone_vertices[v] = gate_cone[net.var_gate[v]];
    return lc;
}

std::vector<int> near_input_select(const Tree &t, const std::vector<Legs> &legs, int n_vars,
                                   const std::vector<char> &forbidden, const LightCones &lc, int k, size_t cone_max) {
    // weight of a variable: summed cost of the contraction steps it indexes
    // (relative to the largest), i.e. how much projecting it saves
    const int ns = (int)t.steps.size();
    std::vector<Legs> un(ns);
    double mxr = 0;
    for (int s = 0; s < ns; s++) {
        un[s] = merge_union(legs[t.steps[s].first], legs[t.steps[s].second]);
        mxr = std::max(mxr, (double)un[s].size());
    }
    std::vector<double> w(n_vars, 0.0);
    for (int s = 0; s < ns; s++) {
        const double c = std::exp2((double)un[s].size() - mxr);
        for (int v : un[s]) w[v] += c;
    }
    std::vector<int> cand;
    for (int v = 0; v < n_vars; v++)
        if (!forbidden[v] && !lc.cone_vertices[v].empty() && lc.cone_vertices[v].size() <= cone_max) cand.push_back(v);
    std::stable_sort(cand.begin(), cand.end(), [&](int a, int b) { return w[a] > w[b]; });
    std::vector<int> S;
    for (int v : cand) {
        if ((int)S.size() >= k) break;
        const Legs &cv = lc.cone_vertices[v];
        bool ok = true;
        for (int u : S) {
            const Legs &cu = lc.cone_vertices[u];
            if (std::binary_search(cv.begin(), cv.end(), u) || std::binary_search(cu.begin(), cu.end(), v)) {
                ok = false;
                break;
            }
        }
        if (ok) S.push_back(v);
    }
    return S;
}

std::vector<int> sliced_vertex_select(const LightCones &lc, const std::vector<int> &I, int k) {
    // Appendix B, SlicedVertexSelect: grow S greedily by the candidate whose
    // addition gives the smallest |L'_C(S u {u})|; candidates exclude the
    // current cover and S itself; members inside the new vertex's cone leave S.
    std::vector<int> S;
    Legs cover;
    Legs Iset(I);
    std::sort(Iset.begin(), Iset.end());
    while ((int)S.size() < k) {
        int best = -1;
        size_t best_sz = 0;
        for (int u : Iset) {
            if (std::binary_search(cover.begin(), cover.end(), u)) continue;
            if (std::find(S.begin(), S.end(), u) != S.end()) continue;
            size_t sz = merge_union(cover, lc.cone_vertices[u]).size();
            if (best < 0 || sz < best_sz) best = u, best_sz = sz;
        }
        if (best < 0) break;
        const Legs &cb = lc.cone_vertices[best];
        std::vector<int> ns;
        for (int s : S)
            if (!std::binary_search(cb.begin(), cb.end(), s)) ns.push_back(s);
        ns.push_back(best);
        S = ns;
        cover.clear();
        for (int s : S) cover = merge_union(cover, lc.cone_vertices[s]);
    }
    std::sort(S.begin(), S.end());
    return S;
}

} // namespace rqc
