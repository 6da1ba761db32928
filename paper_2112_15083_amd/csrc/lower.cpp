// Lowering of a sliced contraction tree to a launch program.
//
// Tensors are complex64 arrays over binary legs; a layout is the list of legs
// from the least significant bit of the element index upwards.  Steps are
// lowered three ways:
//   - subtrees whose tensors all have at most 2^kSmallLog elements run fused,
//     one workgroup per subtree, with their intermediates in LDS (OP_SMALL);
//   - steps with a short contracted dimension, or a thin free dimension, run
//     as a streaming contraction that reads each operand element in place
//     through bit maps (OP_STREAM, bound by HBM bandwidth);
//   - the rest are complex GEMMs on MFMA (OP_GEMM), with operands permuted
//     (OP_PERMUTE) into [batch][rows][cols] form when their layout does not
//     already have it.
// Intermediate buffers share one arena whose offsets come from a first-fit
// plan over their lifetimes.
#include <algorithm>
#include <cmath>
#include <functional>
#include <numeric>
#include <tuple>

#include "host.hpp"

namespace rqc {

static constexpr int kSmallLog = 10;     // largest tensor inside a fused subtree
static constexpr int kLdsBudget = 4096;  // complex64 elements of LDS per fused subtree
static constexpr int kAlign = 64;        // arena alignment in elements (512 bytes)

BitMap make_map(const std::vector<int> &l2m) {
    BitMap m;
    int i = 0;
    const int n = (int)l2m.size();
    while (i < n) {
        if (l2m[i] < 0) {
            i++;
            continue;
        }
        int j = i + 1;
        while (j < n && l2m[j] == l2m[j - 1] + 1) j++;
        if (m.n >= kMaxRuns) fail(RQC_EPLAN, "bit map has too many runs");
        m.run[m.n] = (uint32_t)i | (uint32_t)(j - i) << 8 | (uint32_t)l2m[i] << 16;
        m.n++;
        i = j;
    }
    return m;
}

static int pos_in(const std::vector<int> &layout, int v) {
    for (size_t i = 0; i < layout.size(); i++)
        if (layout[i] == v) return (int)i;
    return -1;
}

static bool contains(const Legs &s, int v) { return std::binary_search(s.begin(), s.end(), v); }

// Does `layout` consist of the groups g0, g1, g2 (as sets), in that order from bit 0?
static bool fits3(const std::vector<int> &layout, const Legs &g0, const Legs &g1, const Legs &g2) {
    size_t i = 0;
    for (const Legs *g : {&g0, &g1, &g2}) {
        for (size_t k = 0; k < g->size(); k++, i++)
            if (i >= layout.size() || !contains(*g, layout[i])) return false;
    }
    return i == layout.size();
}

static std::vector<int> ordered_subset(const std::vector<int> &layout, const Legs &set) {
    std::vector<int> out;
    for (int v : layout)
        if (contains(set, v)) out.push_back(v);
    return out;
}

static Legs set_of(std::vector<int> v) {
    std::sort(v.begin(), v.end());
    return v;
}

struct Lowerer {
    const Tree &tree;
    const std::vector<Legs> &legs;
    Program &prog;
    int nt;
    std::vector<std::vector<int>> layout;
    std::vector<Buf> where;        // location of each tensor once materialised
    std::vector<int> parent;
    std::vector<char> sub_small;   // whole subtree is small-eligible
    std::vector<char> in_small;    // step executed inside a fused subtree (not its root)
    // arena buffers
    struct Alloc {
        int64_t size;
        int first, last; // op indices of production and last use
        int64_t off = -1;
    };
    std::vector<Alloc> allocs;
    std::vector<int> tensor_alloc; // tensor -> alloc index (-1 none)
    std::vector<int> op_first_use;
    int op_counter = 0;
    // global cache: dep[t] = tensor t depends on the fixed output bits
    std::vector<char> dep;
    bool cache = false;
    // fused streaming pairs: deferred[t] = step t runs inside its parent's op
    bool fuse = true;
    std::vector<char> deferred;
    // matrix-core streaming forms allowed (off: vector-ALU kernels only)
    bool mx_streams = true;

    Lowerer(const Tree &t, const std::vector<Legs> &l, Program &p, const std::vector<char> &leaf_dep, bool cache_,
            bool fuse_, bool mx_)
        : tree(t), legs(l), prog(p), cache(cache_), fuse(fuse_ && mx_), mx_streams(mx_) {
        nt = t.n_leaves + (int)t.steps.size();
        layout.resize(nt);
        where.resize(nt);
        parent.assign(nt, -1);
        deferred.assign(nt, 0);
        tensor_alloc.assign(nt, -1);
        dep.assign(nt, 1);
        for (int i = 0; i < t.n_leaves; i++) dep[i] = leaf_dep[i];
        for (size_t s = 0; s < t.steps.size(); s++) {
            parent[t.steps[s].first] = t.n_leaves + (int)s;
            parent[t.steps[s].second] = t.n_leaves + (int)s;
            dep[t.n_leaves + s] = dep[t.steps[s].first] | dep[t.steps[s].second];
        }
        prog.cache = cache;
    }

    // a tensor the per-batch steps read but do not compute: kept in the cache
    bool frontier(int t) const { return cache && !dep[t] && (parent[t] < 0 || dep[parent[t]]); }
    Buf cache_alloc(int64_t size) {
        Buf b;
        b.kind = 2;
        b.off = prog.cache_elems;
        prog.cache_elems += (size + kAlign - 1) / kAlign * kAlign;
        return b;
    }

    int64_t size_of(int t) const { return (int64_t)1 << legs[t].size(); }

    int new_alloc(int64_t size, int tensor) {
        allocs.push_back({size, op_counter, op_counter});
        if (tensor >= 0) tensor_alloc[tensor] = (int)allocs.size() - 1;
        return (int)allocs.size() - 1;
    }
    void touch(int alloc) {
        if (alloc >= 0) allocs[alloc].last = std::max(allocs[alloc].last, op_counter);
    }

    // ---------------------------------------------------------------- small subtrees
    // Emit the steps of the subtree rooted at t (post-order) into prog.small_steps.
    // Returns the LDS offset of the result (or -1 when it is a leaf).  `lds_used`
    // tracks a simple free list over LDS.
    struct Lds {
        std::vector<std::pair<int, int>> blocks; // (offset, size) in use
        int peak = 0;
        int alloc(int size) {
            std::sort(blocks.begin(), blocks.end());
            int off = 0;
            for (auto &b : blocks) {
                if (b.first - off >= size) break;
                off = std::max(off, b.first + b.second);
            }
            blocks.push_back({off, size});
            peak = std::max(peak, off + size);
            return off;
        }
        void release(int off) {
            for (size_t i = 0; i < blocks.size(); i++)
                if (blocks[i].first == off) {
                    blocks.erase(blocks.begin() + i);
                    return;
                }
        }
    };

    int subtree_peak(int t) {
        // LDS elements needed to evaluate t's subtree in post-order (larger child first)
        if (t < tree.n_leaves) return 0;
        auto [a, b] = tree.steps[t - tree.n_leaves];
        int pa = subtree_peak(a), pb = subtree_peak(b);
        int sa = a < tree.n_leaves ? 0 : (int)size_of(a);
        int sb = b < tree.n_leaves ? 0 : (int)size_of(b);
        int first = std::max(pa, pb + sa);
        int second = std::max(pb, pa + sb);
        int kids = std::min(first, second);
        return std::max(kids, sa + sb + (int)size_of(t));
    }

    void emit_small_step(int t, int a_kind, int64_t a_off, int b_kind, int64_t b_off, int c_kind,
                         int64_t c_off) {
        auto [a, b] = tree.steps[t - tree.n_leaves];
        const Legs &C = legs[t];
        std::vector<int> &LA = layout[a], &LB = layout[b];
        // C layout: A's surviving legs in A order, then B's new legs in B order
        std::vector<int> LC;
        for (int v : LA)
            if (contains(C, v)) LC.push_back(v);
        for (int v : LB)
            if (contains(C, v) && pos_in(LA, v) < 0) LC.push_back(v);
        if (c_kind != 0) LC = preferred_layout(t, LC); // a fused subtree's result
        layout[t] = LC;
        std::vector<int> con;
        for (int v : LA)
            if (!contains(C, v) && pos_in(LB, v) >= 0) con.push_back(v);
        SmallStep st;
        st.a_kind = a_kind;
        st.b_kind = b_kind;
        st.c_kind = c_kind;
        st.a_off = a_off;
        st.b_off = b_off;
        st.c_off = c_off;
        st.rc = (int)LC.size();
        st.kc = (int)con.size();
        std::vector<int> ax(LC.size()), bx(LC.size()), ay(con.size()), by(con.size());
        for (size_t j = 0; j < LC.size(); j++) ax[j] = pos_in(LA, LC[j]), bx[j] = pos_in(LB, LC[j]);
        for (size_t j = 0; j < con.size(); j++) ay[j] = pos_in(LA, con[j]), by[j] = pos_in(LB, con[j]);
        st.ax = make_map(ax);
        st.bx = make_map(bx);
        st.ay = make_map(ay);
        st.by = make_map(by);
        prog.small_steps.push_back(st);
        double f = 8.0 * std::exp2((double)(LC.size() + con.size()));
        prog.flops += f;
    }

    // returns (kind, offset) of where t's value sits during the subtree program
    std::pair<int, int64_t> eval_small(int t, Lds &lds, bool is_root) {
        if (t < tree.n_leaves) return {1, where[t].off};
        auto [a, b] = tree.steps[t - tree.n_leaves];
        int pa = subtree_peak(a), pb = subtree_peak(b);
        int sa = a < tree.n_leaves ? 0 : (int)size_of(a);
        int sb = b < tree.n_leaves ? 0 : (int)size_of(b);
        bool a_first = std::max(pa, pb + sa) <= std::max(pb, pa + sb);
        std::pair<int, int64_t> ra, rb;
        if (a_first) {
            ra = eval_small(a, lds, false);
            rb = eval_small(b, lds, false);
        } else {
            rb = eval_small(b, lds, false);
            ra = eval_small(a, lds, false);
        }
        int ck;
        int64_t co;
        if (is_root) {
            ck = 2;
            co = -1; // patched once the arena buffer exists
        } else {
            ck = 0;
            co = lds.alloc((int)size_of(t));
        }
        emit_small_step(t, ra.first, ra.second, rb.first, rb.second, ck, co);
        if (ra.first == 0) lds.release((int)ra.second);
        if (rb.first == 0) lds.release((int)rb.second);
        return {ck, co};
    }

    void mark_sub_small() {
        sub_small.assign(nt, 0);
        for (int i = 0; i < tree.n_leaves; i++) sub_small[i] = legs[i].size() <= (size_t)kSmallLog;
        for (size_t s = 0; s < tree.steps.size(); s++) {
            int t = tree.n_leaves + (int)s;
            auto [a, b] = tree.steps[s];
            sub_small[t] = sub_small[a] && sub_small[b] && legs[t].size() <= (size_t)kSmallLog;
        }
        // enforce the LDS budget: a small subtree too big for LDS is cut below
        for (int t = nt - 1; t >= tree.n_leaves; t--) {
            if (!sub_small[t]) continue;
            bool root = parent[t] < 0 || !sub_small[parent[t]];
            if (root && subtree_peak(t) > kLdsBudget) {
                // evaluate the children as their own fused subtrees
                sub_small[t] = 0;
            }
        }
        // repeat until stable (cutting a node exposes its children as roots)
        bool changed = true;
        while (changed) {
            changed = false;
            for (int t = nt - 1; t >= tree.n_leaves; t--) {
                if (!sub_small[t]) continue;
                bool root = parent[t] < 0 || !sub_small[parent[t]];
                if (root && subtree_peak(t) > kLdsBudget) {
                    sub_small[t] = 0;
                    changed = true;
                }
            }
        }
    }

    // ---------------------------------------------------------------- phase-2 steps
    Buf buf_of(int t) { return where[t]; }

    void use_tensor(int t) {
        if (tensor_alloc[t] >= 0) touch(tensor_alloc[t]);
    }

    Buf materialise(int t) {
        if (frontier(t)) {
            where[t] = cache_alloc(size_of(t));
            return where[t];
        }
        int al = new_alloc(size_of(t), t);
        Buf b;
        b.kind = 0;
        b.off = al; // resolved to an element offset after the arena plan
        where[t] = b;
        return b;
    }

    // Legs of tensor t that its consumer keeps as batch legs (in both operands
    // and in the result) when that consumer is a streaming step.  Streaming
    // tiles run over non-batch legs, so t keeps these legs at its high
    // positions and leaves its low (contiguous) positions to legs a tile covers.
    // When that consumer runs fused with its own consumer, the batch legs of
    // either step cannot be tile rows either (unless the second step
    // contracts them), so they go high too.
    Legs late_legs(int t) {
        Legs out;
        const int par = parent[t];
        if (par < 0 || gemm_worthy(par)) return out;
        auto [a, b] = tree.steps[par - tree.n_leaves];
        const Legs &o = legs[a == t ? b : a], &pc = legs[par];
        for (int v : legs[t])
            if (contains(o, v) && contains(pc, v)) out.push_back(v);
        if (par >= tree.n_leaves && !in_small[par] && fusable(par) && step_legs(par).a == t) {
            const StepLegs s2 = step_legs(parent[par]);
            for (int v : legs[t])
                if (contains(s2.q, v) && !contains(s2.k, v) && !contains(out, v)) out.push_back(v);
            Legs keep;
            for (int v : out)
                if (!contains(s2.k, v)) keep.push_back(v);
            std::sort(keep.begin(), keep.end());
            out = keep;
        }
        return out;
    }
    static std::vector<int> late_last(std::vector<int> v, const Legs &late) {
        std::stable_partition(v.begin(), v.end(), [&](int x) { return !contains(late, x); });
        return v;
    }

    // Layout of a computed tensor whose natural layout is LC.  With a GEMM
    // consumer: one of that GEMM's operand layouts (A: [K | M | batch] or
    // [M | K | batch], B: [N | K | batch] or [K | N | batch]), so no permute is
    // needed.  The contracted and batch groups stay ascending (the other
    // operand uses the same orders); the free group follows LC, with the legs
    // that the GEMM's own streaming consumer batches over last; and the
    // free-group-first form is taken when its low legs agree better with LC's,
    // which keeps the producing step's reads and writes contiguous together.
    // Otherwise LC with the consumer's batch legs last.
    std::vector<int> preferred_layout(int t, const std::vector<int> &LC) {
        const int par = parent[t];
        if (par >= 0 && gemm_worthy(par)) {
            auto [pa, pb] = tree.steps[par - tree.n_leaves];
            const Legs &PA = legs[pa], &PB = legs[pb], &PC = legs[par];
            Legs bt, cn, fa_, fb_;
            for (int v : PA) {
                bool inb = contains(PB, v), inc = contains(PC, v);
                if (inb && inc) bt.push_back(v);
                else if (inb) cn.push_back(v);
                else fa_.push_back(v);
            }
            for (int v : PB)
                if (!contains(PA, v)) fb_.push_back(v);
            std::vector<int> fr(t == pa ? fa_ : fb_);
            std::stable_sort(fr.begin(), fr.end(), [&](int x, int y) { return pos_in(LC, x) < pos_in(LC, y); });
            fr = late_last(fr, late_legs(par));
            std::vector<int> kf = cn, ff = fr; // contracted group first / free group first
            kf.insert(kf.end(), fr.begin(), fr.end());
            ff.insert(ff.end(), cn.begin(), cn.end());
            kf.insert(kf.end(), bt.begin(), bt.end());
            ff.insert(ff.end(), bt.begin(), bt.end());
            if (set_of(kf) != legs[t]) return LC;
            // low legs shared with LC (a streaming tile spans at most 11 bits)
            const size_t T = std::min<size_t>(11, LC.size());
            auto agree = [&](const std::vector<int> &W) {
                int n = 0;
                for (size_t j = 0; j < T; j++)
                    n += std::find(LC.begin(), LC.begin() + T, W[j]) != LC.begin() + T;
                return n;
            };
            // B's default is free group first ([N | K]), A's contracted first
            const bool free_first = t == pa ? agree(ff) > agree(kf) : agree(ff) >= agree(kf);
            return free_first ? ff : kf;
        }
        return late_last(LC, late_legs(t));
    }

    // A streaming step's operands (large one first) and result layout: the
    // large operand's order with its contracted legs replaced in place by the
    // new legs, then the consumer's preferences (preferred_layout).
    void stream_layout(int t, int &a, int &b, std::vector<int> &LC, std::vector<int> &con,
                       std::vector<int> &newb) {
        std::tie(a, b) = tree.steps[t - tree.n_leaves];
        if (size_of(b) > size_of(a)) std::swap(a, b);
        const Legs &C = legs[t];
        const std::vector<int> &LA = layout[a], &LB = layout[b];
        newb.clear(), LC.clear(), con.clear();
        for (int v : LB)
            if (contains(C, v) && pos_in(LA, v) < 0) newb.push_back(v);
        size_t nb = 0;
        for (int v : LA) {
            if (contains(C, v))
                LC.push_back(v);
            else {
                con.push_back(v);
                if (nb < newb.size()) LC.push_back(newb[nb++]);
            }
        }
        for (; nb < newb.size(); nb++) LC.push_back(newb[nb]);
        LC = preferred_layout(t, LC);
    }

    // Leg classes of a streaming step t (operands a = large, b): contracted k,
    // new f, batch q (in both operands and the result), rows (A and result).
    struct StepLegs {
        int a, b;
        Legs k, f, q, rows;
    };
    StepLegs step_legs(int t) {
        StepLegs s;
        std::tie(s.a, s.b) = tree.steps[t - tree.n_leaves];
        if (size_of(s.b) > size_of(s.a)) std::swap(s.a, s.b);
        const Legs &A = legs[s.a], &B = legs[s.b], &C = legs[t];
        for (int v : A) {
            if (!contains(C, v)) s.k.push_back(v);
            else {
                s.rows.push_back(v);
                if (contains(B, v)) s.q.push_back(v);
            }
        }
        for (int v : B)
            if (contains(C, v) && !contains(A, v)) s.f.push_back(v);
        return s;
    }

    // Can streaming step t1 run fused into its consumer (k_stream_mx2)?  The
    // consumer streams t1's result with t1 as its large operand; the first
    // step contracts 2^4 or 2^5 and adds 2^5, the second contracts 2^4 legs
    // that are rows of the first (at most two of them batch legs of the first)
    // and adds 2^4; the second step's batch legs are rows of the first outside
    // the tile; and both steps run in the same cache phase.
    bool fusable(int t1) {
        if (!fuse) return false;
        const int t2 = parent[t1];
        if (t2 < 0 || in_small[t2] || gemm_worthy(t2)) return false;
        const StepLegs s1 = step_legs(t1), s2 = step_legs(t2);
        if (s2.a != t1) return false;
        // (a first step adding 2^4 legs also fits the kernel, but halves the
        // work per tile behind the same barriers: measured no faster than the
        // two steps apart, so such pairs stay separate)
        if ((s1.k.size() != 4 && s1.k.size() != 5) || s1.f.size() != 5 || s2.k.size() != 4 || s2.f.size() != 4)
            return false;
        if (dep[t1] != dep[t2]) return false;
        int kq = 0;
        for (int v : s2.k) {
            if (!contains(s1.rows, v)) return false;
            kq += contains(s1.q, v);
        }
        if (kq > 2) return false;
        for (int v : s2.q)
            if (contains(s1.f, v)) return false;
        int extra = 0;
        for (int v : s1.rows)
            extra += !contains(s2.k, v) && !contains(s1.q, v) && !contains(s2.q, v);
        return extra >= 2 && s1.rows.size() >= 8;
    }

    // Legs of t that a fused pair further up contracts, when t reaches that
    // pair's large operand through one GEMM (whose output keeps the order of
    // t's free legs): t keeps them first among its low legs, so that the
    // pair's tile covers the low positions of its large operand.
    Legs early_legs(int t) {
        Legs out;
        const int g = parent[t];
        if (g < 0 || !gemm_worthy(g)) return out;
        const int s = parent[g];
        if (s < 0 || in_small[s] || gemm_worthy(s) || !fusable(s) || step_legs(s).a != g) return out;
        const StepLegs u1 = step_legs(s), u2 = step_legs(parent[s]);
        for (int v : legs[t])
            if (contains(u1.k, v) || contains(u2.k, v)) out.push_back(v);
        return out;
    }

    // Number of C's lowest positions (layout LC of tensor t) that the tile of
    // a fused pair whose large operand is t would cover: the pair's contracted
    // legs and, as in emit_fused, the two lowest rows that neither step
    // batches over nor the second contracts.  0 when t is not such an operand.
    int pair_tile_prefix(int t, const std::vector<int> &LC) {
        const int p1 = parent[t];
        if (p1 < 0 || in_small[p1] || gemm_worthy(p1) || !fusable(p1) || step_legs(p1).a != t) return 0;
        const StepLegs u1 = step_legs(p1), u2 = step_legs(parent[p1]);
        int n = 0, rows = 0;
        for (int v : LC) {
            if (contains(u1.k, v) || contains(u2.k, v)) n++;
            else if (rows < 2 && contains(u1.rows, v) && !contains(u1.q, v) && !contains(u2.q, v)) n++, rows++;
            else break;
        }
        return n;
    }

    // A GEMM whose result is a fused pair's large operand writes its output
    // [M | N] with N lowest.  When N's lowest legs give the pair's tile fewer
    // than four low bits (a 128-byte line), two tiles share every line and the
    // operand is read twice.  If the first M legs are legs the pair contracts,
    // putting them right after that N prefix lengthens the tile's run: returns
    // how many M legs to insert (0: leave [M | N]).
    int pair_tile_insert(int t, const std::vector<int> &fbord, const std::vector<int> &faord) {
        std::vector<int> LC = fbord;
        LC.insert(LC.end(), faord.begin(), faord.end());
        const int s0 = pair_tile_prefix(t, LC);
        if (s0 == 0 || s0 >= 4 || s0 >= (int)fbord.size()) return 0;
        const int p1 = parent[t];
        const StepLegs u1 = step_legs(p1), u2 = step_legs(parent[p1]);
        for (int ins = 1; ins <= 3 && ins <= (int)faord.size(); ins++) {
            const int v = faord[ins - 1];
            if (!contains(u1.k, v) && !contains(u2.k, v)) return 0;
            std::vector<int> W(fbord.begin(), fbord.begin() + s0);
            W.insert(W.end(), faord.begin(), faord.begin() + ins);
            W.insert(W.end(), fbord.begin() + s0, fbord.end());
            W.insert(W.end(), faord.begin() + ins, faord.end());
            if (pair_tile_prefix(t, W) >= 4) return ins;
        }
        return 0;
    }

    // Emit the fused op for the pair (t1 -> t2); false if its tiles do not
    // allow the kernel's 16-byte accesses (then both steps run separately).
    bool emit_fused(int t1, int t2) {
        const StepLegs s1 = step_legs(t1), s2 = step_legs(t2);
        const std::vector<int> &LA1 = layout[s1.a], &LB1 = layout[s1.b], &LB2 = layout[s2.b];
        // tile rows: the two lowest legs of A1 that neither step batches over
        // nor the second contracts, then the second step's contracted legs,
        // those that index B1 last
        std::vector<int> ext;
        for (int v : LA1)
            if (contains(s1.rows, v) && !contains(s2.k, v) && !contains(s1.q, v) && !contains(s2.q, v))
                ext.push_back(v);
        std::vector<int> T(ext.begin(), ext.begin() + 2);
        for (int v : s2.k)
            if (!contains(s1.q, v)) T.push_back(v);
        for (int v : s2.k)
            if (contains(s1.q, v)) T.push_back(v);
        // outer rows: batch legs of either step first (a workgroup's tiles then
        // share B1 and B2), then the rest by A1 position
        std::vector<int> outer;
        for (int v : LA1)
            if (contains(s1.rows, v) && std::find(T.begin(), T.end(), v) == T.end() &&
                (contains(s1.q, v) || contains(s2.q, v)))
                outer.push_back(v);
        for (int v : LA1)
            if (contains(s1.rows, v) && std::find(T.begin(), T.end(), v) == T.end() &&
                !(contains(s1.q, v) || contains(s2.q, v)))
                outer.push_back(v);
        std::vector<int> rows = T;
        rows.insert(rows.end(), outer.begin(), outer.end());
        // C2's layout: the output tile's legs (the two extra legs, the first
        // step's new legs, the second's) lowest, then the outer rows in A1
        // order, before the consumer's preferences
        std::vector<int> LC2(T.begin(), T.begin() + 2);
        for (int v : LB1)
            if (contains(s1.f, v)) LC2.push_back(v);
        for (int v : LB2)
            if (contains(s2.f, v)) LC2.push_back(v);
        {   // within the tile's legs, those a fused pair further up contracts first
            const Legs early = early_legs(t2);
            std::stable_partition(LC2.begin(), LC2.end(), [&](int v) { return contains(early, v); });
        }
        LC2.insert(LC2.end(), outer.begin(), outer.end());
        LC2 = preferred_layout(t2, LC2);
        // index orders: y1 by A1 position, f1 and f2 by C2 position
        std::vector<int> y1;
        for (int v : LA1)
            if (contains(s1.k, v)) y1.push_back(v);
        std::vector<int> f1(s1.f.begin(), s1.f.end()), f2(s2.f.begin(), s2.f.end());
        auto by_c2 = [&](int x, int y) { return pos_in(LC2, x) < pos_in(LC2, y); };
        std::sort(f1.begin(), f1.end(), by_c2);
        std::sort(f2.begin(), f2.end(), by_c2);
        auto positions = [&](const std::vector<int> &layout_, const std::vector<int> &ls) {
            std::vector<int> out(ls.size());
            for (size_t j = 0; j < ls.size(); j++) out[j] = pos_in(layout_, ls[j]);
            return out;
        };
        StreamOp op;
        op.mx2 = 1;
        op.tile_l = 6;
        op.nr = (int)rows.size();
        op.kc = (int)s1.k.size();
        op.nf = (int)s1.f.size();
        op.kc2 = 4;
        op.nf2 = 4;
        op.rc = (int)LC2.size();
        op.m[SM_RA] = make_map(positions(LA1, rows));
        op.m[SM_RB] = make_map(positions(LB1, rows));
        op.m[SM_YB] = make_map(positions(LB1, y1));
        op.m[SM_FB] = make_map(positions(LB1, f1));
        std::vector<int> rb2 = positions(LB2, rows);
        for (int i = 0; i < 6; i++) rb2[i] = -1; // B2's contracted legs go through YB2
        op.m[SM_RB2] = make_map(rb2);
        op.m[SM_YB2] = make_map(positions(LB2, std::vector<int>(T.begin() + 2, T.end())));
        op.m[SM_FB2] = make_map(positions(LB2, f2));
        std::vector<int> rc = positions(LC2, rows);
        for (int i = 0; i < 6; i++) rc[i] = -1; // the tile's legs: in the C2 tile, or contracted
        op.m[SM_RC] = make_map(rc);
        auto idx = [](const std::vector<int> &P, int pos) {
            return (int)(std::lower_bound(P.begin(), P.end(), pos) - P.begin());
        };
        // A1 tile: (six tile rows, contracted legs) by A1 position
        std::vector<int> PA;
        for (int i = 0; i < 6; i++) PA.push_back(pos_in(LA1, rows[i]));
        for (int v : y1) PA.push_back(pos_in(LA1, v));
        std::sort(PA.begin(), PA.end());
        std::vector<int> er(PA.size()), ey(PA.size());
        for (int i = 0; i < 6; i++) er[idx(PA, pos_in(LA1, rows[i]))] = i, ey[idx(PA, pos_in(LA1, rows[i]))] = -1;
        for (size_t j = 0; j < y1.size(); j++) ey[idx(PA, pos_in(LA1, y1[j]))] = (int)j, er[idx(PA, pos_in(LA1, y1[j]))] = -1;
        op.m[SM_EA] = make_map(PA);
        op.m[SM_ER] = make_map(er);
        op.m[SM_EY] = make_map(ey);
        // C2 tile: rows r' = (two extra legs, f1), new legs f2, by C2 position
        std::vector<int> rp = {T[0], T[1]};
        rp.insert(rp.end(), f1.begin(), f1.end());
        std::vector<int> PC;
        for (int v : rp) PC.push_back(pos_in(LC2, v));
        for (int v : f2) PC.push_back(pos_in(LC2, v));
        std::sort(PC.begin(), PC.end());
        std::vector<int> er2(PC.size()), ef(PC.size());
        for (size_t i = 0; i < rp.size(); i++) er2[idx(PC, pos_in(LC2, rp[i]))] = (int)i, ef[idx(PC, pos_in(LC2, rp[i]))] = -1;
        for (size_t j = 0; j < f2.size(); j++) ef[idx(PC, pos_in(LC2, f2[j]))] = (int)j, er2[idx(PC, pos_in(LC2, f2[j]))] = -1;
        op.m[SM_EC] = make_map(PC);
        op.m[SM_ER2] = make_map(er2);
        op.m[SM_EF] = make_map(ef);
        // 16-byte accesses: tile bit 0 is tensor bit 0 on both sides, spans at
        // 32-bit byte offsets
        int64_t spanA = 0, spanC = 0;
        for (int v : PA) spanA += (int64_t)1 << v;
        for (int v : PC) spanC += (int64_t)1 << v;
        if (PA[0] != 0 || PC[0] != 0 || spanA >= ((int64_t)1 << 29) || spanC >= ((int64_t)1 << 29)) return false;
        // commit: the pair's operands, and its result in t2's place
        layout[t2] = LC2;
        op.a = buf_of(s1.a);
        op.b = buf_of(s1.b);
        op.b2 = buf_of(s2.b);
        use_tensor(s1.a);
        use_tensor(s1.b);
        use_tensor(s2.b);
        op.c = materialise(t2);
        const double f = 8.0 * (std::exp2((double)(s1.rows.size() + s1.k.size() + s1.f.size())) +
                                std::exp2((double)(s2.rows.size() + s2.k.size() + s2.f.size())));
        const double by_ = 8.0 * (double)(size_of(s1.a) + size_of(s1.b) + size_of(s2.b) + size_of(t2));
        prog.streams.push_back(op);
        prog.ops.push_back({OP_STREAM, (int)prog.streams.size() - 1, f, by_, dep[t2]});
        if (!dep[t2]) prog.flops_indep += f;
        prog.flops += f;
        prog.bytes += by_;
        op_counter++;
        return true;
    }

    void emit_stream(int t) {
        // a step that can run inside its consumer's op waits for it
        if (!deferred[t] && fusable(t)) {
            int a, b;
            std::vector<int> LC, con, newb;
            stream_layout(t, a, b, LC, con, newb);
            layout[t] = LC;
            deferred[t] = 1;
            return;
        }
        {
            auto [a0, b0] = tree.steps[t - tree.n_leaves];
            const int big = size_of(b0) > size_of(a0) ? b0 : a0;
            if (big >= tree.n_leaves && deferred[big] == 1) {
                if (emit_fused(big, t)) return;
                deferred[big] = 2; // not fused after all: run it first
                emit_stream(big);
            }
        }
        auto [a, b] = tree.steps[t - tree.n_leaves];
        if (size_of(b) > size_of(a)) std::swap(a, b);
        const Legs &C = legs[t];
        const std::vector<int> &LA = layout[a], &LB = layout[b];
        std::vector<int> LC, con, newb;
        {
            int a_, b_;
            stream_layout(t, a_, b_, LC, con, newb);
        }
        (void)C;
        layout[t] = LC;
        StreamOp op;
        op.a = buf_of(a);
        op.b = buf_of(b);
        use_tensor(a);
        use_tensor(b);
        op.c = materialise(t);
        op.rc = (int)LC.size();
        op.kc = (int)con.size();
        std::vector<int> rest, fpos;
        for (size_t j = 0; j < LC.size(); j++)
            (std::find(newb.begin(), newb.end(), LC[j]) != newb.end() ? fpos : rest).push_back((int)j);
        op.nr = (int)rest.size();
        op.nf = (int)fpos.size();
        // A tile is the first L kept legs with all contracted and new legs.  The
        // kept legs go lowest first by their lower position in A or C, so that a
        // tile's reads and writes both run over the low positions of their
        // tensors even when C's layout does not follow A's.
        // (six new legs: tiles of 2^12 C elements and 64 rows, matrix-core form only)
        const int L = op.kc <= 5 && op.nf == 6 && op.nr >= 6 ? 6
                      : (op.kc <= 5 && op.nf <= 10) ? std::min({op.nr, 11 - std::max(op.kc, op.nf), 8}) : 0;
        if (L > 0) {
            std::stable_sort(rest.begin(), rest.end(), [&](int x, int y) {
                const int kx = std::min(pos_in(LA, LC[x]), x), ky = std::min(pos_in(LA, LC[y]), y);
                return kx != ky ? kx < ky : pos_in(LA, LC[x]) < pos_in(LA, LC[y]);
            });
        }
        // Matrix-core form: order the tile's legs non-batch first, so that a
        // quarter tile (one wave's rows) shares one B matrix, then the other
        // batch legs, so that a workgroup's successive tiles share one too.
        auto is_batch = [&](int j) { return pos_in(LB, LC[j]) >= 0; };
        // At most two batch legs fit a tile (they are its top row bits); further
        // ones are passed over for the next non-batch legs, which costs some
        // contiguity of the tile but keeps the step on the matrix cores.
        if (mx_streams && L >= 6 && op.kc <= 5 && op.nf <= 6) {
            std::vector<int> tile;
            int nbt = 0;
            for (size_t i = 0; i < rest.size() && (int)tile.size() < L; i++)
                if (!is_batch(rest[i]) || nbt < 2) tile.push_back(rest[i]), nbt += is_batch(rest[i]);
            if ((int)tile.size() == L) {
                op.mx = 1;
                std::vector<int> r2;
                for (int j : tile)
                    if (!is_batch(j)) r2.push_back(j);
                for (int j : tile)
                    if (is_batch(j)) r2.push_back(j);
                auto in_tile = [&](int j) { return std::find(tile.begin(), tile.end(), j) != tile.end(); };
                for (int j : rest)
                    if (!in_tile(j) && is_batch(j)) r2.push_back(j);
                for (int j : rest)
                    if (!in_tile(j) && !is_batch(j)) r2.push_back(j);
                rest = r2;
            }
        }
        // Long contraction on matrix cores: 64 rows per workgroup from six
        // non-batch kept legs (lowest A positions first), 32-wide chunks of the
        // contracted index from its five legs with the lowest A positions.
        if (mx_streams && L == 0 && op.kc >= 6 && op.nf <= 5) {
            std::vector<int> nbr;
            for (int j : rest)
                if (!is_batch(j)) nbr.push_back(j);
            if (nbr.size() >= 6) {
                op.lk = 1;
                std::stable_sort(nbr.begin(), nbr.end(),
                                 [&](int x, int y) { return pos_in(LA, LC[x]) < pos_in(LA, LC[y]); });
                std::vector<int> r2(nbr.begin(), nbr.begin() + 6);
                for (int j : rest)
                    if (std::find(r2.begin(), r2.end(), j) == r2.end()) r2.push_back(j);
                rest = r2;
                std::stable_sort(con.begin(), con.end(), [&](int x, int y) { return pos_in(LA, x) < pos_in(LA, y); });
            }
        }
        std::vector<int> ra(rest.size()), rb(rest.size()), rcm(rest.size()), fb(fpos.size()), fc(fpos.size());
        for (size_t j = 0; j < rest.size(); j++) {
            ra[j] = pos_in(LA, LC[rest[j]]);
            rb[j] = pos_in(LB, LC[rest[j]]);
            rcm[j] = rest[j];
        }
        for (size_t j = 0; j < fpos.size(); j++) fb[j] = pos_in(LB, LC[fpos[j]]), fc[j] = fpos[j];
        std::vector<int> ay(con.size()), by(con.size());
        for (size_t j = 0; j < con.size(); j++) ay[j] = pos_in(LA, con[j]), by[j] = pos_in(LB, con[j]);
        op.m[SM_RA] = make_map(ra);
        op.m[SM_RB] = make_map(rb);
        op.m[SM_RC] = make_map(rcm);
        op.m[SM_FB] = make_map(fb);
        op.m[SM_FC] = make_map(fc);
        op.m[SM_YA] = make_map(ay);
        op.m[SM_YB] = make_map(by);
        if (op.lk) {
            std::vector<int> PA, PB;
            for (int i = 0; i < 6; i++) PA.push_back(ra[i]);
            for (int j = 0; j < 5; j++) PA.push_back(ay[j]), PB.push_back(by[j]);
            for (int v : fb) PB.push_back(v);
            std::sort(PA.begin(), PA.end());
            std::sort(PB.begin(), PB.end());
            std::vector<int> er(PA.size(), -1), ey(PA.size(), -1), bY(PB.size(), -1), bF(PB.size(), -1);
            auto idx = [](const std::vector<int> &P, int pos) {
                return (int)(std::lower_bound(P.begin(), P.end(), pos) - P.begin());
            };
            for (int i = 0; i < 6; i++) er[idx(PA, ra[i])] = i;
            for (int j = 0; j < 5; j++) ey[idx(PA, ay[j])] = j, bY[idx(PB, by[j])] = j;
            for (size_t j = 0; j < fb.size(); j++) bF[idx(PB, fb[j])] = (int)j;
            op.m[SM_EA] = make_map(PA);
            op.m[SM_ER] = make_map(er);
            op.m[SM_EY] = make_map(ey);
            op.m[SM_EB] = make_map(PB);
            op.m[SM_BY] = make_map(bY);
            op.m[SM_BF] = make_map(bF);
            // unsplit: the workgroup's 64 x 2^nf outputs go to C through LDS, in
            // C's memory order (tile element -> C offset, row, new index)
            std::vector<int> PC;
            for (int i = 0; i < 6; i++) PC.push_back(rcm[i]);
            for (int v : fc) PC.push_back(v);
            std::sort(PC.begin(), PC.end());
            std::vector<int> er2(PC.size(), -1), ef(PC.size(), -1);
            for (int i = 0; i < 6; i++) er2[idx(PC, rcm[i])] = i;
            for (size_t j = 0; j < fc.size(); j++) ef[idx(PC, fc[j])] = (int)j;
            op.m[SM_EC] = make_map(PC);
            op.m[SM_ER2] = make_map(er2);
            op.m[SM_EF] = make_map(ef);
            // about 2048 workgroups: 2^(nr-6) row groups times the chunk splits
            op.lk_split = std::max(0, std::min(op.kc - 5, 11 - (op.nr - 6)));
            if (op.lk_split > 0) {
                op.w.kind = 0;
                op.w.off = new_alloc((int64_t)1 << (op.lk_split + op.nr + op.nf), -1);
            }
        }
        // LDS tiling when both the contracted and the new-leg dimensions are
        // short: tiles hold at most 2^11 elements of A and of C, and at most 256
        // rows (one per thread of the register-blocked form)
        if (L >= 1) {
            op.tile_l = L;
            std::vector<int> PA, PC;
            for (int i = 0; i < L; i++) PA.push_back(ra[i]), PC.push_back(rcm[i]);
            for (int v : ay) PA.push_back(v);
            for (int v : fc) PC.push_back(v);
            std::sort(PA.begin(), PA.end());
            std::sort(PC.begin(), PC.end());
            auto idx = [](const std::vector<int> &P, int pos) {
                return (int)(std::lower_bound(P.begin(), P.end(), pos) - P.begin());
            };
            std::vector<int> re(L), ye(ay.size()), re2(L), fe(fc.size());
            for (int i = 0; i < L; i++) re[i] = idx(PA, ra[i]), re2[i] = idx(PC, rcm[i]);
            for (size_t j = 0; j < ay.size(); j++) ye[j] = idx(PA, ay[j]);
            for (size_t j = 0; j < fc.size(); j++) fe[j] = idx(PC, fc[j]);
            op.m[SM_EA] = make_map(PA);
            op.m[SM_RE] = make_map(re);
            op.m[SM_YE] = make_map(ye);
            op.m[SM_EC] = make_map(PC);
            op.m[SM_RE2] = make_map(re2);
            op.m[SM_FE] = make_map(fe);
            // row-major staging for the matrix-core form: tile element -> row / index
            std::vector<int> er(PA.size(), -1), ey(PA.size(), -1), er2(PC.size(), -1), ef(PC.size(), -1);
            for (int i = 0; i < L; i++) er[re[i]] = i, er2[re2[i]] = i;
            for (size_t j = 0; j < ay.size(); j++) ey[ye[j]] = (int)j;
            for (size_t j = 0; j < fc.size(); j++) ef[fe[j]] = (int)j;
            op.m[SM_ER] = make_map(er);
            op.m[SM_EY] = make_map(ey);
            op.m[SM_ER2] = make_map(er2);
            op.m[SM_EF] = make_map(ef);
            // the matrix-core kernel moves pairs of adjacent elements (tile bit 0
            // must be tensor bit 0) at 32-bit offsets from the tile base: bytes, or
            // elements in the wide form
            if (op.mx) {
                int64_t spanA = 0, spanC = 0;
                for (int v : PA) spanA += (int64_t)1 << v;
                for (int v : PC) spanC += (int64_t)1 << v;
                if (PA[0] != 0 || PC[0] != 0 || spanA >= ((int64_t)1 << 32) || spanC >= ((int64_t)1 << 32))
                    op.mx = 0;
                // past 4 GiB of byte offsets: element offsets and 64-bit addresses
                op.wide = spanA >= ((int64_t)1 << 29) || spanC >= ((int64_t)1 << 29);
            }
            if (!op.mx && L + op.nf > 11) op.tile_l = -1; // too large for the vector tile kernel
        }
        double f = 8.0 * std::exp2((double)(LC.size() + con.size()));
        double by_ = 8.0 * (double)(size_of(a) + size_of(b) + size_of(t));
        prog.streams.push_back(op);
        (void)set_of;
        prog.ops.push_back({OP_STREAM, (int)prog.streams.size() - 1, f, by_, dep[t]});
        if (!dep[t]) prog.flops_indep += f;
        prog.flops += f;
        prog.bytes += by_;
        op_counter++;
    }

    // permute tensor t into `target` layout; returns the new buffer
    Buf emit_permute(int t, const std::vector<int> &target) {
        PermuteOp op;
        op.src = buf_of(t);
        use_tensor(t);
        op.r = (int)target.size();
        op.perm.resize(op.r);
        for (int i = 0; i < op.r; i++) op.perm[i] = pos_in(target, layout[t][i]);
        // the permuted copy of a cached tensor is what the per-batch steps read
        int al = -1;
        if (frontier(t)) {
            op.dst = cache_alloc(size_of(t));
        } else {
            al = new_alloc(size_of(t), -1);
            op.dst.kind = 0;
            op.dst.off = al;
        }
        double by_ = 16.0 * (double)size_of(t);
        prog.permutes.push_back(op);
        prog.ops.push_back({OP_PERMUTE, (int)prog.permutes.size() - 1, 0.0, by_, dep[t]});
        prog.bytes += by_;
        op_counter++;
        perm_alloc_last = al;
        return op.dst;
    }
    int perm_alloc_last = -1;

    void emit_gemm(int t) {
        auto [a, b] = tree.steps[t - tree.n_leaves];
        const Legs &A = legs[a], &B = legs[b], &C = legs[t];
        Legs batch, con, fa, fb;
        for (int v : A) {
            bool inb = contains(B, v), inc = contains(C, v);
            if (inb && inc) batch.push_back(v);
            else if (inb) con.push_back(v);
            else if (inc) fa.push_back(v);
            else fail(RQC_EPLAN, "leg summed within one operand");
        }
        for (int v : B)
            if (!contains(A, v)) {
                if (contains(C, v)) fb.push_back(v);
                else fail(RQC_EPLAN, "leg summed within one operand");
            }
        const std::vector<int> &LA = layout[a], &LB = layout[b];
        // A view
        int a_kfast;
        std::vector<int> kord, bord, faord, fbord;
        bool a_ok = true;
        if (fits3(LA, con, fa, batch)) a_kfast = 1;
        else if (fits3(LA, fa, con, batch)) a_kfast = 0;
        else a_ok = false, a_kfast = 1;
        kord = ordered_subset(LA, con);
        bord = ordered_subset(LA, batch);
        faord = ordered_subset(LA, fa);
        fbord = ordered_subset(LB, fb);
        // C's lowest legs are B's free legs: those a streaming consumer batches
        // over go last, permuting B for it when B is small
        bool fb_moved = false;
        if (const Legs late = late_legs(t); !late.empty()) {
            std::vector<int> w = late_last(fbord, late);
            if (w != fbord && size_of(b) <= ((int64_t)1 << 24)) fbord = w, fb_moved = true;
        }
        // B view with A's K and batch orders
        auto b_layout = [&](int nfast) {
            std::vector<int> L;
            if (nfast) {
                L = fbord;
                L.insert(L.end(), kord.begin(), kord.end());
            } else {
                L = kord;
                L.insert(L.end(), fbord.begin(), fbord.end());
            }
            L.insert(L.end(), bord.begin(), bord.end());
            return L;
        };
        int b_nfast = -1;
        if (LB == b_layout(1)) b_nfast = 1;
        else if (LB == b_layout(0)) b_nfast = 0;
        // If B fits its own groups but in a different K/batch order, consider
        // permuting A to B's orders instead when A is the smaller tensor.
        if (b_nfast < 0 && !fb_moved && size_of(a) < size_of(b)) {
            bool bk = fits3(LB, fb, con, batch), bn = fits3(LB, con, fb, batch);
            if (bk || bn) {
                kord = ordered_subset(LB, con);
                bord = ordered_subset(LB, batch);
                b_nfast = bk ? 1 : 0;
                a_ok = false; // A will be permuted to match
                a_kfast = 1;
            }
        }
        Buf abuf = buf_of(a), bbuf = buf_of(b);
        int a_tmp = -1, b_tmp = -1;
        std::vector<int> LAt;
        if (a_kfast) {
            LAt = kord;
            LAt.insert(LAt.end(), faord.begin(), faord.end());
        } else {
            LAt = faord;
            LAt.insert(LAt.end(), kord.begin(), kord.end());
        }
        LAt.insert(LAt.end(), bord.begin(), bord.end());
        if (!a_ok || LAt != LA) {
            abuf = emit_permute(a, LAt);
            a_tmp = perm_alloc_last;
        }
        if (b_nfast < 0) {
            b_nfast = 1;
            bbuf = emit_permute(b, b_layout(1));
            b_tmp = perm_alloc_last;
        }
        GemmOp g;
        g.a = abuf;
        g.b = bbuf;
        use_tensor(a);
        use_tensor(b);
        if (a_tmp >= 0) touch(a_tmp);
        if (b_tmp >= 0) touch(b_tmp);
        g.batch = (int64_t)1 << batch.size();
        g.M = (int64_t)1 << fa.size();
        g.N = (int64_t)1 << fb.size();
        g.K = (int64_t)1 << con.size();
        g.a_kfast = a_kfast;
        g.b_nfast = b_nfast;
        g.c_nfast = 1;
        g.sa = g.M * g.K;
        g.sb = g.K * g.N;
        g.sc = g.M * g.N;
        // when the output tiles (the launcher's 128 or 64 a side) cannot fill
        // the chip, split K into ranges of at least 128 whose partial sums go
        // to scratch and are added in range order
        {
            const int64_t tiles = g.batch * (g.M / (g.M >= 128 ? 128 : 64)) * (g.N / (g.N >= 128 ? 128 : 64));
            int ks = 1;
            while (tiles * ks < 1024 && g.K / (2 * ks) >= 128) ks *= 2;
            if (ks > 1) {
                g.ksplit = ks;
                g.w.kind = 0;
                g.w.off = new_alloc((int64_t)ks * g.batch * g.M * g.N, -1);
            }
        }
        std::vector<int> LC = fbord;
        LC.insert(LC.end(), faord.begin(), faord.end());
        LC.insert(LC.end(), bord.begin(), bord.end());
        if (const int ins = pair_tile_insert(t, fbord, faord); ins > 0) {
            // the first `ins` M legs go between N legs so that a fused pair's
            // tile covers C's lowest 16-byte-line bits (see pair_tile_insert)
            const int s0 = pair_tile_prefix(t, LC);
            std::vector<int> W(fbord.begin(), fbord.begin() + s0);
            W.insert(W.end(), faord.begin(), faord.begin() + ins);
            W.insert(W.end(), fbord.begin() + s0, fbord.end());
            W.insert(W.end(), faord.begin() + ins, faord.end());
            W.insert(W.end(), bord.begin(), bord.end());
            LC = W;
            g.c_ins_pos = s0;
            g.c_ins_bits = ins;
        }
        layout[t] = LC;
        g.c = materialise(t);
        if (a_tmp >= 0) touch(a_tmp);
        if (b_tmp >= 0) touch(b_tmp);
        double f = 8.0 * (double)g.batch * (double)g.M * (double)g.N * (double)g.K;
        double by_ = 8.0 * (double)g.batch * (double)(g.M * g.K + g.K * g.N + g.M * g.N);
        prog.gemms.push_back(g);
        prog.ops.push_back({OP_GEMM, (int)prog.gemms.size() - 1, f, by_, dep[t]});
        if (!dep[t]) prog.flops_indep += f;
        prog.flops += f;
        prog.gemm_flops += f;
        prog.bytes += by_;
        op_counter++;
    }

    bool gemm_worthy(int t) {
        auto [a, b] = tree.steps[t - tree.n_leaves];
        const Legs &A = legs[a], &B = legs[b], &C = legs[t];
        int nb = 0, nk = 0, nfa = 0, nfb = 0;
        for (int v : A) {
            bool inb = contains(B, v), inc = contains(C, v);
            if (inb && inc) nb++;
            else if (inb) nk++;
            else nfa++;
        }
        for (int v : B)
            if (!contains(A, v)) nfb++;
        (void)nb;
        return nk >= 3 && nfa >= 6 && nfb >= 6;
    }

    void run(const std::vector<int> &leaf_offsets) {
        for (int i = 0; i < tree.n_leaves; i++) {
            layout[i] = legs[i]; // sorted, as produced by the leaf-select kernel
            where[i].kind = 1;
            where[i].off = leaf_offsets[i];
        }
        mark_sub_small();
        // fused small subtrees: roots are small steps whose parent is not small
        in_small.assign(nt, 0);
        // fused small subtrees, those that do not depend on the fixed bits first
        std::vector<int> small_roots;
        for (int pass = 0; pass < 2; pass++)
            for (int t = tree.n_leaves; t < nt; t++)
                if (sub_small[t] && (parent[t] < 0 || !sub_small[parent[t]]) && dep[t] == pass) small_roots.push_back(t);
        for (int t : small_roots) {
            Lds lds;
            int first = (int)prog.small_steps.size();
            const double f0 = prog.flops;
            eval_small(t, lds, true);
            if (!dep[t]) prog.flops_indep += prog.flops - f0;
            SmallTree st;
            st.first_step = first;
            st.n_steps = (int)prog.small_steps.size() - first;
            prog.small_trees.push_back(st);
            prog.small_lds_elems = std::max(prog.small_lds_elems, lds.peak);
            Buf out = materialise(t);
            prog.small_steps.back().c_off = out.off; // alloc index, resolved below
            if (out.kind == 2) prog.small_steps.back().c_kind = 3;
            if (!dep[t]) prog.n_small_indep++;
            // mark inner steps
            std::function<void(int)> mark = [&](int u) {
                if (u < tree.n_leaves) return;
                in_small[u] = 1;
                mark(tree.steps[u - tree.n_leaves].first);
                mark(tree.steps[u - tree.n_leaves].second);
            };
            mark(t);
        }
        if (!prog.small_trees.empty()) {
            double by_ = 0;
            for (auto &s : prog.small_trees) {
                (void)s;
            }
            prog.ops.push_back({OP_SMALL, 0, 0.0, by_});
            op_counter++;
        }
        // remaining steps in tree order
        for (int t = tree.n_leaves; t < nt; t++) {
            if (in_small[t]) continue;
            if (gemm_worthy(t)) emit_gemm(t);
            else emit_stream(t);
        }
        int root = tree.root();
        use_tensor(root);
        op_counter++;
        // arena plan: first fit by decreasing size over lifetime overlaps
        std::vector<int> order(allocs.size());
        std::iota(order.begin(), order.end(), 0);
        std::sort(order.begin(), order.end(), [&](int x, int y) {
            return allocs[x].size != allocs[y].size ? allocs[x].size > allocs[y].size : x < y;
        });
        std::vector<int> placed;
        int64_t extent = 0;
        for (int i : order) {
            Alloc &al = allocs[i];
            int64_t sz = (al.size + kAlign - 1) / kAlign * kAlign;
            std::vector<std::pair<int64_t, int64_t>> busy;
            for (int j : placed) {
                const Alloc &o = allocs[j];
                if (o.first <= al.last && al.first <= o.last)
                    busy.push_back({o.off, o.off + (o.size + kAlign - 1) / kAlign * kAlign});
            }
            std::sort(busy.begin(), busy.end());
            int64_t off = 0;
            for (auto &b : busy) {
                if (b.first - off >= sz) break;
                off = std::max(off, b.second);
            }
            al.off = off;
            extent = std::max(extent, off + sz);
            placed.push_back(i);
        }
        prog.arena_elems = extent;
        auto fix = [&](Buf &b) {
            if (b.kind == 0) b.off = allocs[b.off].off;
        };
        for (auto &s : prog.small_steps)
            if (s.c_kind == 2) s.c_off = allocs[s.c_off].off; // cache offsets (kind 3) are final
        for (auto &s : prog.streams) {
            fix(s.a), fix(s.b), fix(s.c);
            if (s.mx2) fix(s.b2);
            if (s.lk && s.lk_split > 0) fix(s.w);
        }
        for (auto &p : prog.permutes) fix(p.src), fix(p.dst);
        for (auto &g : prog.gemms) {
            fix(g.a), fix(g.b), fix(g.c);
            if (g.ksplit > 1) fix(g.w);
        }
        for (int t = 0; t < nt; t++)
            if (where[t].kind == 0 && tensor_alloc[t] >= 0) where[t].off = allocs[tensor_alloc[t]].off;
        prog.root = where[root];
        for (int t = 0; t < nt; t++) prog.max_log2 = std::max(prog.max_log2, (int)legs[t].size());
    }
};

int stream_kernel(const StreamOp &op) {
    if (op.mx2) return SK_MX2;
    if (op.mx) return SK_MX;
    if (op.lk) return SK_LK;
    if (op.tile_l < 0 && op.kc >= 6 && op.nf <= 4) return SK_KY;
    if (op.tile_l >= 0) return SK_TILE;
    return SK_GEN;
}

// Lower the tree.  leaf_offsets: element offset of each projected leaf in the
// leaf buffer.  Returns the root layout through `root_layout`.
Program lower_tree(const Tree &tree, const std::vector<Legs> &legs, const std::vector<int> &leaf_offsets,
                   const std::vector<char> &leaf_dep, bool cache, bool fuse, bool mx_streams,
                   std::vector<int> &root_layout) {
    Program prog;
    Lowerer L(tree, legs, prog, leaf_dep, cache, fuse, mx_streams);
    L.run(leaf_offsets);
    root_layout = L.layout[tree.root()];
    return prog;
}

} // namespace rqc
