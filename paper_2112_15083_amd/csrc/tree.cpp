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

namespace {
struct Cand {
    double key;
    int a, b;
    bool operator<(const Cand &o) const { return key > o.key; } // min-heap
};
} // namespace

Tree greedy_tree(const std::vector<Legs> &leaf_legs, int n_vars, const std::vector<char> &kept,
                 uint64_t seed, double temperature) {
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
        double sc = std::exp2((double)out_legs(a, b).size()) - std::exp2((double)legs[a].size()) -
                    std::exp2((double)legs[b].size());
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
