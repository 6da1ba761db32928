// Simulated annealing of the contraction tree T and the sliced variables I.
//
// Sec. I of the paper takes T and I as the inputs of the method and optimises
// them by simulated annealing; the moves and the cost are not described there,
// so the ones below are this library's:
//   * tree moves: at an internal node u = (x, y) with y = (y0, y1), exchange x
//     with one of y's children, u' = (y_{1-j}, (x, y_j)).  Only the node that
//     takes y's place and u change cost; u keeps its leaf set and its legs;
//   * slicing moves: exchange a sliced leg with an unsliced leg of one of the
//     largest tensors, and, when no leg count is prescribed, drop a sliced leg
//     or add one;
//   * cost: log2 of the sum over steps of the time-like step cost (complex
//     multiply-adds plus five per element moved, as the greedy search scores
//     trees, plus a fixed launch cost for every step too large for the fused
//     small-subtree launch: without it the moves split the work into hundreds
//     of tiny launches) with the sliced legs removed, plus |I| (the number of
//     slices);
//     every state keeps each tensor within the memory bound;
//   * Metropolis acceptance at a temperature (in log2 units of the total) that
//     falls geometrically from 0.01 to 1e-5 over the iterations: most moves
//     change one small step and barely move the total, so a hotter start lets
//     the small steps drift upwards without bound; the best state seen is
//     returned.
// Leg sets are bitsets over the variables; a tensor's legs follow from its
// subtree's occurrence set: after the move, the legs of y' = (x, y_j) are
// (occ(x) | occ(y_j)) & (legs(u) | occ(y_{1-j}) | kept).
#include <algorithm>
#include <cmath>
#include <random>

#include "host.hpp"

namespace rqc {

namespace {

class Annealer {
  public:
    Annealer(const Tree &t, const std::vector<int> &sliced, const std::vector<Legs> &leaf_legs, int n_vars,
             const std::vector<char> &kept, const std::vector<char> &forbidden, int max_log2, bool slice_moves,
             int n_target, uint64_t seed)
        : L(t.n_leaves), ns((int)t.steps.size()), nt(L + ns), W((n_vars + 63) / 64), nv(n_vars), M(max_log2),
          slicing(slice_moves), target(n_target), forb(forbidden), rng(seed) {
        ca.assign(nt, -1);
        cb.assign(nt, -1);
        par.assign(nt, -1);
        for (int s = 0; s < ns; s++) {
            const int u = L + s;
            ca[u] = t.steps[s].first;
            cb[u] = t.steps[s].second;
            par[ca[u]] = par[cb[u]] = u;
        }
        root = t.root();
        occ.assign((size_t)nt * W, 0);
        lg.assign((size_t)nt * W, 0);
        keptb.assign(W, 0);
        slb.assign(W, 0);
        scratch_occ.assign(W, 0);
        scratch_lg.assign(W, 0);
        for (int v = 0; v < nv; v++)
            if (kept[v]) keptb[v >> 6] |= 1ull << (v & 63);
        for (int v : sliced) slb[v >> 6] |= 1ull << (v & 63), in_I.push_back(v);
        // occurrence sets bottom-up (SSA order); legs(u) = occ(u) & (occurrence
        // outside u's subtree | kept), the outside sets from the top down
        for (int i = 0; i < L; i++)
            for (int v : leaf_legs[i]) occ[(size_t)i * W + (v >> 6)] |= 1ull << (v & 63);
        for (int s = 0; s < ns; s++) {
            const int u = L + s;
            for (int w = 0; w < W; w++)
                occ[(size_t)u * W + w] = occ[(size_t)ca[u] * W + w] | occ[(size_t)cb[u] * W + w];
        }
        std::vector<uint64_t> out((size_t)nt * W, 0);
        for (int u = nt - 1; u >= L; u--) {
            const int a = ca[u], b = cb[u];
            for (int w = 0; w < W; w++) {
                out[(size_t)a * W + w] = out[(size_t)u * W + w] | occ[(size_t)b * W + w];
                out[(size_t)b * W + w] = out[(size_t)u * W + w] | occ[(size_t)a * W + w];
            }
        }
        for (int u = 0; u < nt; u++)
            for (int w = 0; w < W; w++)
                lg[(size_t)u * W + w] = occ[(size_t)u * W + w] & (out[(size_t)u * W + w] | keptb[w]);
        recompute();
    }

    // Run `iters` moves; returns the best (tree, sliced, log2 cost) seen.
    SearchResult run(int iters) {
        save_best();
        if (ns < 2) return best_result();
        std::uniform_real_distribution<double> U(0.0, 1.0);
        const double T0 = 0.01, T1 = 1e-5;
        for (int it = 0; it < iters; it++) {
            const double T = T0 * std::pow(T1 / T0, (double)it / std::max(1, iters - 1));
            if (slicing && !in_I.empty() && U(rng) < 0.1) slice_move(T, U(rng));
            else tree_move(T);
            if (objective() < best_obj - 1e-12) save_best();
            if ((it & 4095) == 4095) recompute(); // no drift in the running sum
        }
        return best_result();
    }

  private:
    int L, ns, nt, W, nv, M, root;
    bool slicing;
    int target;
    const std::vector<char> &forb;
    std::mt19937_64 rng;
    std::vector<int> ca, cb, par;
    std::vector<uint64_t> occ, lg, keptb, slb;
    std::vector<uint64_t> scratch_occ, scratch_lg; // a move's candidate leg sets
    std::vector<int> in_I;
    std::vector<double> cost; // per internal node
    double total = 0;
    // best state
    std::vector<int> bca, bcb, bI;
    int broot = 0;
    double best_obj = 1e300;

    const uint64_t *L_(int u) const { return &lg[(size_t)u * W]; }
    const uint64_t *O_(int u) const { return &occ[(size_t)u * W]; }

    int rank_of(const uint64_t *a) const {
        int r = 0;
        for (int w = 0; w < W; w++) r += __builtin_popcountll(a[w] & ~slb[w]);
        return r;
    }
    int rank_union(const uint64_t *a, const uint64_t *b) const {
        int r = 0;
        for (int w = 0; w < W; w++) r += __builtin_popcountll((a[w] | b[w]) & ~slb[w]);
        return r;
    }
    double node_cost(int u) const {
        return step_time_cost(rank_of(L_(ca[u])), rank_of(L_(cb[u])), rank_union(L_(ca[u]), L_(cb[u])),
                              rank_of(L_(u)), true);
    }
    void recompute() {
        cost.assign(nt, 0.0);
        total = 0;
        for (int u = L; u < nt; u++) total += cost[u] = node_cost(u);
    }
    double objective() const { return std::log2(std::max(total, 1.0)) + (double)in_I.size(); }

    void tree_move(double T) {
        std::uniform_int_distribution<int> pick(L, nt - 1);
        const int u = pick(rng);
        int side = (int)(rng() & 1);
        int y = side ? cb[u] : ca[u];
        if (y < L) {
            side ^= 1;
            y = side ? cb[u] : ca[u];
            if (y < L) return;
        }
        const int x = side ? ca[u] : cb[u];
        const int j = (int)(rng() & 1);
        const int yj = j ? cb[y] : ca[y], yk = j ? ca[y] : cb[y];
        // legs of y' = (x, y_j)
        uint64_t *nocc = scratch_occ.data(), *nlg = scratch_lg.data();
        for (int w = 0; w < W; w++) {
            nocc[w] = O_(x)[w] | O_(yj)[w];
            nlg[w] = nocc[w] & (L_(u)[w] | O_(yk)[w] | keptb[w]);
        }
        const int r_new = rank_of(nlg);
        if (M > 0 && r_new > M) return;
        const double c_y = step_time_cost(rank_of(L_(x)), rank_of(L_(yj)), rank_union(L_(x), L_(yj)), r_new, true);
        const double c_u = step_time_cost(rank_of(L_(yk)), r_new, rank_union(L_(yk), nlg), rank_of(L_(u)), true);
        const double nt_total = total - cost[y] - cost[u] + c_y + c_u;
        const double d = std::log2(std::max(nt_total, 1.0)) - std::log2(std::max(total, 1.0));
        if (d > 0 && std::uniform_real_distribution<double>(0.0, 1.0)(rng) >= std::exp2(-d / T)) return;
        // apply: y becomes (x, y_j), u becomes (y_k, y)
        ca[y] = x;
        cb[y] = yj;
        par[x] = y;
        par[yj] = y;
        ca[u] = yk;
        cb[u] = y;
        par[yk] = u;
        par[y] = u;
        for (int w = 0; w < W; w++) occ[(size_t)y * W + w] = nocc[w], lg[(size_t)y * W + w] = nlg[w];
        cost[y] = c_y;
        cost[u] = c_u;
        total = nt_total;
    }

    bool has(const uint64_t *a, int v) const { return (a[v >> 6] >> (v & 63)) & 1; }

    // total cost and largest rank with v unsliced (remove >= 0) and w sliced (add >= 0)
    std::pair<double, int> eval_slicing(int remove, int add) const {
        double t = 0;
        int mx = 0;
        auto adj = [&](const uint64_t *a, int r) {
            if (remove >= 0 && has(a, remove)) r++;
            if (add >= 0 && has(a, add)) r--;
            return r;
        };
        std::vector<int> rk(nt);
        for (int u = 0; u < nt; u++) {
            rk[u] = adj(L_(u), rank_of(L_(u)));
            mx = std::max(mx, rk[u]);
        }
        for (int u = L; u < nt; u++) {
            int ru = rank_union(L_(ca[u]), L_(cb[u]));
            if (remove >= 0 && (has(L_(ca[u]), remove) || has(L_(cb[u]), remove))) ru++;
            if (add >= 0 && (has(L_(ca[u]), add) || has(L_(cb[u]), add))) ru--;
            t += step_time_cost(rk[ca[u]], rk[cb[u]], ru, rk[u], true);
        }
        return {t, mx};
    }

    // an unsliced, sliceable leg of one of the largest tensors
    int pick_add() {
        int mx = 0;
        std::vector<int> big;
        for (int u = L; u < nt; u++) {
            const int r = rank_of(L_(u));
            if (r > mx) mx = r, big.clear();
            if (r == mx) big.push_back(u);
        }
        if (big.empty()) return -1;
        const int u = big[rng() % big.size()];
        std::vector<int> c;
        for (int v = 0; v < nv; v++)
            if (has(L_(u), v) && !has(slb.data(), v) && !forb[v] && !has(keptb.data(), v)) c.push_back(v);
        return c.empty() ? -1 : c[rng() % c.size()];
    }

    void slice_move(double T, double kind) {
        int remove = -1, add = -1;
        const bool fixed_count = target >= 0;
        if (fixed_count || kind < 0.5) {
            remove = in_I[rng() % in_I.size()];
            add = pick_add();
            if (add < 0) return;
        } else if (kind < 0.75) {
            remove = in_I[rng() % in_I.size()];
        } else {
            add = pick_add();
            if (add < 0) return;
        }
        auto [t, mx] = eval_slicing(remove, add);
        if (M > 0 && mx > M) return;
        const int dI = (add >= 0) - (remove >= 0);
        const double d = std::log2(std::max(t, 1.0)) + dI - std::log2(std::max(total, 1.0));
        if (d > 0 && std::uniform_real_distribution<double>(0.0, 1.0)(rng) >= std::exp2(-d / T)) return;
        if (remove >= 0) {
            slb[remove >> 6] &= ~(1ull << (remove & 63));
            in_I.erase(std::find(in_I.begin(), in_I.end(), remove));
        }
        if (add >= 0) {
            slb[add >> 6] |= 1ull << (add & 63);
            in_I.push_back(add);
        }
        recompute();
    }

    void save_best() {
        best_obj = objective();
        bca = ca;
        bcb = cb;
        broot = root;
        bI = in_I;
    }

    SearchResult best_result() const {
        // SSA order: post-order from the root
        SearchResult r;
        r.tree.n_leaves = L;
        std::vector<int> id(nt, -1);
        for (int i = 0; i < L; i++) id[i] = i;
        std::vector<int> stack{broot};
        std::vector<char> done(nt, 0);
        while (!stack.empty()) {
            const int u = stack.back();
            if (u < L) {
                stack.pop_back();
                continue;
            }
            if (!done[u]) {
                done[u] = 1;
                stack.push_back(bca[u]);
                stack.push_back(bcb[u]);
            } else {
                stack.pop_back();
                id[u] = L + (int)r.tree.steps.size();
                r.tree.steps.push_back({id[bca[u]], id[bcb[u]]});
            }
        }
        r.sliced = bI;
        r.log2cost = best_obj;
        return r;
    }
};

} // namespace

SearchResult anneal_tree(const Tree &t, const std::vector<int> &sliced, const std::vector<Legs> &leaf_legs,
                         int n_vars, const std::vector<char> &kept, const std::vector<char> &forbidden,
                         int max_log2_tensor, bool slice_moves, int n_target, int iters, uint64_t seed) {
    Annealer a(t, sliced, leaf_legs, n_vars, kept, forbidden, max_log2_tensor, slice_moves, n_target, seed);
    return a.run(iters);
}

} // namespace rqc
