// Internal host-side structures of librqc: circuit, hyper tensor network,
// contraction tree, slicing and the lowered launch program.
#pragma once

#include <complex>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "rqc.h"

namespace rqc {

using cf = std::complex<float>;
using cd = std::complex<double>;

struct Error {
    rqc_status code;
    std::string msg;
};
[[noreturn]] void fail(rqc_status code, const std::string &msg);

// ------------------------------------------------------------------ circuit
enum GateKind { G_SX = 0, G_SY = 1, G_SW = 2, G_FSIM = 3 };

struct Gate {
    int kind = 0;
    int q[2] = {-1, -1};
    long tnum = 0, tden = 1; // theta / pi
    long pnum = 0, pden = 1; // phi / pi
    bool swap_like() const { return kind == G_FSIM && 2 * tnum == tden; }
};

struct Circuit {
    int n = 0;
    std::vector<Gate> gates;
};

Circuit parse_circuit(const char *text, size_t len);

// ------------------------------------------------------------------ network
// One tensor per gate line.  Variables follow the numbering of rqc.h.
struct Leaf {
    std::vector<int> legs; // variable ids; legs[0] is bit 0 of the element index
    std::vector<cf> data;  // 2^legs.size() values (input variables already fixed to 0)
    double scale = 1.0;    // data = scale * (exact tensor), up to complex64 rounding
};

struct Network {
    int n_qubits = 0;
    int n_vars = 0;
    std::vector<Leaf> leaves;
    std::vector<int> out_var;       // per qubit: variable on that wire at the end
    std::vector<int> var_gate;      // creating gate line (-1 for inputs)
    std::vector<std::vector<int>> gate_inputs; // input variables of each gate line
};

Network build_network(const Circuit &c);

// ------------------------------------------------------------------ tree
using Legs = std::vector<int>; // sorted variable ids

struct Tree {
    int n_leaves = 0;
    std::vector<std::pair<int, int>> steps; // SSA operand ids; step s creates n_leaves + s
    int root() const { return steps.empty() ? 0 : n_leaves + (int)steps.size() - 1; }
};

// Leg sets of every tensor of the tree (leaves then steps) for a given set of
// removed (projected) variables and kept (never summed) variables.
std::vector<Legs> tree_legs(const Tree &t, const std::vector<Legs> &leaf_legs, int n_vars,
                            const std::vector<char> &removed, const std::vector<char> &kept);

double tree_log2_cost_sum(const Tree &t, const std::vector<Legs> &legs); // log2 sum 2^|A u B|

Tree greedy_tree(const std::vector<Legs> &leaf_legs, int n_vars, const std::vector<char> &kept,
                 uint64_t seed, double temperature, double costmod = 1.0);

// Re-optimise every subtree of up to `k` frontier tensors exactly (dynamic
// programming over subsets), minimising flops plus written elements.
Tree reconfigure_tree(const Tree &t, const std::vector<Legs> &leaf_legs, int n_vars,
                      const std::vector<char> &kept, int k, int passes);

std::vector<int> greedy_slice(const Tree &t, const std::vector<Legs> &legs, int n_vars,
                              const std::vector<char> &forbidden, int max_log2_tensor,
                              int n_target);

// Randomised greedy trials (temperature and size weighting drawn per trial),
// each followed by subtree reconfiguration and slicing; the trial with the
// smallest total sliced cost wins.  Trials run on host threads.
struct SearchResult {
    Tree tree;
    std::vector<int> sliced;
    double log2cost = 0;
};
// Time-like cost of one pairwise step of ranks ra, rb (operands), runion
// (their union) and rc (result): multiply-adds plus weighted elements moved,
// plus a fixed launch cost for unfused steps when `launches`.
double step_time_cost(int ra, int rb, int runion, int rc, bool launches = false);
// Simulated annealing of a tree and its sliced legs (anneal.cpp): `iters`
// Metropolis moves from (t, sliced); slicing moves only if slice_moves (and
// keeping |sliced| when n_target >= 0); every state within max_log2_tensor.
SearchResult anneal_tree(const Tree &t, const std::vector<int> &sliced, const std::vector<Legs> &leaf_legs,
                         int n_vars, const std::vector<char> &kept, const std::vector<char> &forbidden,
                         int max_log2_tensor, bool slice_moves, int n_target, int iters, uint64_t seed);
// The reconfigured best trials (a sixteenth of `trials`, at least 8), best proxy cost first.
std::vector<SearchResult> search_tree(const std::vector<Legs> &leaf_legs, int n_vars, const std::vector<char> &kept,
                                      const std::vector<char> &forbidden, const std::vector<int> *user_sliced,
                                      int max_log2_tensor, int n_target, int trials, uint64_t seed);

// ------------------------------------------------------------------ light cones (Appendix B)
struct LightCones {
    // per variable: sorted list of vertices L'_C(v) (inputs of the gates v depends on)
    std::vector<std::vector<int>> cone_vertices;
};
LightCones light_cones(const Network &net);
std::vector<int> sliced_vertex_select(const LightCones &lc, const std::vector<int> &I, int k);
// Sec. I.B step 1: up to k vertices as close to the inputs as possible (light
// cone of at most cone_max vertices), pairwise outside each other's cones (so
// that they lie on one cut of the circuit), chosen by how much of tree t's
// contraction cost they index (largest first; ties by ascending id).
std::vector<int> near_input_select(const Tree &t, const std::vector<Legs> &legs, int n_vars,
                                   const std::vector<char> &forbidden, const LightCones &lc, int k, size_t cone_max);

// ------------------------------------------------------------------ lowered program
enum OpKind { OP_SMALL = 0, OP_STREAM = 1, OP_PERMUTE = 2, OP_GEMM = 3 };

// Bit map from a logical index to an element offset: sum over runs of
// ((x >> src) & (2^len - 1)) << dst.  Runs are packed in 32-bit words
// (src | len << 8 | dst << 16) so that device code reads a map with scalar
// loads when the map is the same for the whole wave.
constexpr int kMaxRuns = 24;
struct BitMap {
    int32_t n = 0;
    uint32_t run[kMaxRuns] = {};
    int src(int i) const { return (int)(run[i] & 255u); }
    int len(int i) const { return (int)((run[i] >> 8) & 255u); }
    int dst(int i) const { return (int)(run[i] >> 16); }
};
BitMap make_map(const std::vector<int> &logical_to_mem); // entry = memory bit of logical bit, -1 = absent

struct Buf {      // where a tensor lives
    int kind = 0; // 0 = arena, 1 = projected-leaf buffer, 2 = global cache (per slice group)
    int64_t off = 0; // element offset (complex64 elements)
};

struct SmallStep { // one contraction inside a fused small subtree
    int a_kind, b_kind, c_kind; // 0 = LDS, 1 = leaf buffer, 2 = arena, 3 = global cache (root output)
    int64_t a_off, b_off, c_off;
    int rc, kc;                 // log2 |C|, log2 K
    BitMap ax, bx, ay, by;      // C-index -> A/B offsets, K-index -> A/B offsets
};

struct SmallTree {
    int first_step, n_steps;
};

// C[x] = sum_y A[ax(x)+ay(y)] * B[bx(x)+by(y)].  The C index x splits into
// the bits of B's new legs (f, nf bits) and the rest (r, nr bits):
// x = xC(r) + fC(f), A offset = rA(r) + yA(y), B offset = rB(r) + fB(f) + yB(y).
// Tiled form: a tile is 2^tile_l consecutive r; its A operands are the
// 2^(tile_l+kc) elements e (bits: the A positions of r's low bits and of y, in
// ascending order), staged through LDS: A offset = rA(r0) + EA(e), tile slot of
// (r, y) = RE(r_low) + YE(y); outputs likewise with C offset = rC(r0) + EC(e'),
// slot of (r, f) = RE2(r_low) + FE(f).
// Matrix-core form (mx): the same tiles, staged row-major instead: tile element
// e holds row ER(e) and contracted index EY(e) (A side), or row ER2(e) and new
// index EF(e) (C side).  The tile's batch legs (r bits that also index B) are
// its top row bits, so all rows of a quarter tile share one B matrix.
// Long form (lk, 2^kc >= 64): a workgroup takes 64 rows (the first six r bits,
// none of them batch legs) and a range of 32-wide chunks of the contracted
// index (its first five bits); A chunks are staged like tiles (EA / ER / EY),
// B chunks through EB (element -> B offset), BY and BF (element -> y, f).
// Chunk ranges (2^lk_split of them) write partial sums to a scratch buffer w
// laid out [split][r][f], summed afterwards in split order.
// Fused pair (mx2): a streaming step whose large operand is the result of the
// step before it, C2 = (A1 B1) B2, with the intermediate kept in LDS.  The
// first step's tile is 64 rows r (six legs of A1: two extra legs, then the
// second step's four contracted legs, whose batch legs for B1 come last) by
// all its contracted and new legs; it is the k_stream_mx tile (EA, ER, EY,
// RA, RB, YB, FB as there, nr / kc / nf of the first step).  The second step
// takes the tile's 2^(2 + nf) rows r' = (extra legs, first step's new legs)
// and contracts its index y2 = the four tile bits above the extra legs with B2
// (YB2, FB2; RB2 gives B2's offset from the outer row bits, which hold all of
// B2's batch legs).  Its output tile (r', f2) goes to C2 through EC, ER2, EF
// (element -> C2 offset, r', f2) at RC (outer row bits -> C2 offset).
enum {
    SM_RA = 0, SM_RB, SM_RC, SM_FB, SM_FC, SM_YA, SM_YB, SM_EA, SM_RE, SM_YE, SM_EC, SM_RE2, SM_FE,
    SM_ER, SM_EY, SM_ER2, SM_EF, SM_EB, SM_BY, SM_BF, SM_RB2, SM_YB2, SM_FB2, SM_COUNT
};
struct StreamOp {
    Buf a, b, c;
    Buf w;           // lk: partial sums
    int rc, kc, nr, nf;
    int tile_l = -1; // >= 0: tiled kernel with 2^tile_l r per tile
    int mx = 0;      // 1: matrix-core tiled kernel
    int wide = 0;    // mx: a tile spans 2^29 elements or more (64-bit addressed form)
    int lk = 0;      // 1: matrix-core long-contraction kernel
    int lk_split = 0;
    int mx2 = 0;     // 1: fused pair (then b2 is B2, kc2 / nf2 the second step's)
    Buf b2;
    int kc2 = 0, nf2 = 0;
    BitMap m[SM_COUNT];
};

// The kernel a streaming op runs on (launch_stream dispatches on this, and the
// plan report counts it): fused pair, matrix-core tile, matrix-core long
// contraction, then the vector-ALU forms: long contraction, LDS tile, generic.
enum StreamKernel { SK_MX2 = 0, SK_MX, SK_LK, SK_KY, SK_TILE, SK_GEN, SK_COUNT };
int stream_kernel(const StreamOp &op);

struct PermuteOp {  // dst[pi(x)] = src[x]
    Buf src, dst;
    int r;
    std::vector<int> perm; // perm[i] = destination bit of source bit i
};

struct GemmOp {     // C[b][m][n] = sum_k A[b][m][k] B[b][k][n] (complex)
    Buf a, b, c;
    int64_t batch, M, N, K;
    int a_kfast;    // A element (m,k) at m*K + k if 1, k*M + m if 0
    int b_nfast;    // B element (k,n) at k*N + n if 1, n*K + k if 0
    int c_nfast;    // C element (m,n) at m*N + n if 1, n*M + m if 0
    int64_t sa, sb, sc; // batch strides (elements)
    int ksplit = 1; // > 1: K in ksplit ranges, partial sums in w ([range][batch][m][n]), added in order
    Buf w;
    // C's layout with the c_ins_bits low M bits placed between N bits
    // c_ins_pos - 1 and c_ins_pos (0 bits: plain [m][n])
    int c_ins_pos = 0, c_ins_bits = 0;
};

struct Op {
    int kind;
    int index; // into the per-kind arrays
    double flops, bytes;
    int dep = 1; // output depends on the fixed output bits (0: computed once per slice group when cached)
};

// Leaf selection: copy a leaf's sub-tensor with its projected legs fixed.
struct LeafSel {
    int64_t src;          // offset of the full leaf in the leaf store (complex64 elements)
    int64_t dst;          // offset of the projected leaf in the leaf buffer
    int32_t n_free;       // legs kept
    int32_t n_proj;       // legs fixed by projected values
    uint8_t free_pos[4];  // full-layout bit of kept leg j
    uint8_t proj_pos[4];  // full-layout bit of projected leg j
    int16_t proj_idx[4];  // projected-variable index of projected leg j
};

struct Program {
    std::vector<SmallStep> small_steps;
    std::vector<SmallTree> small_trees;
    int small_lds_elems = 0;
    std::vector<StreamOp> streams;
    std::vector<PermuteOp> permutes;
    std::vector<GemmOp> gemms;
    std::vector<Op> ops; // launch order (OP_SMALL appears once, first)
    // global cache: subtrees that do not depend on the fixed output bits; their
    // outputs read by dependent steps live in a per-slice-group cache block
    bool cache = false;
    int n_small_indep = 0;   // small subtrees [0, n) do not depend on fixed bits
    int64_t cache_elems = 0; // per slice group
    double flops_indep = 0;  // per slice group
    // final tensor
    Buf root;
    BitMap root_open, root_slice; // open-batch index / batched-slice index -> offset
    int n_batched = 0;
    int64_t arena_elems = 0;
    int64_t leafbuf_elems = 0;
    double flops = 0, bytes = 0, gemm_flops = 0;
    int max_log2 = 0;
};

// ------------------------------------------------------------------ planning
// A network to plan: its leaves, the legs left open in the result (bit b of
// the result index is open_vars[b]), legs fixed per batch (value = bit
// fixed_bit[i] of the batch's mask) and legs that must not be sliced.
struct NetSpec {
    std::vector<Leaf> leaves;
    int n_vars = 0;
    std::vector<int> open_vars;
    std::vector<int> fixed_vars, fixed_bit;
    std::vector<char> forbidden;
};

NetSpec circuit_spec(const Network &net, const std::vector<int> &open_qubits);
// Doubled network C_1 C_1^* of Fig. 1 for the partially sliced vertices S:
// C_1 = union of the light cones of S; S legs are shared by both copies and
// left open, the other outputs of C_1 are shared and summed.  Its result is
// R[i] = ||psi_i||^2 (Sec. I.A), bit t of i = value of S[t].
NetSpec doubled_spec(const Network &net, const std::vector<int> &S);
void sort_leaf(Leaf &L);

struct PlanCore {
    rqc_plan_opts opts{};
    NetSpec spec;
    Tree tree;
    std::vector<int> sliced, batched, looped;  // variable ids
    std::vector<int> looped_bit, batched_bit;  // bit position of each in a slice id
    bool user_legs = false;                    // sliced legs given by the caller (order kept)
    std::vector<int> S;                        // partially sliced vertices (ascending)
    std::vector<uint64_t> X;                   // kept partial indices, in selection order
    std::vector<double> R;
    double F = 1.0;
    double kappa = 1.0;                        // product of 1/leaf.scale (applied in FP64 at the end)
    std::vector<uint64_t> groups;              // default slice groups: looped-leg values
    uint64_t n_group_range = 0;                // if non-zero: the default groups are 0 .. n-1
    Program prog;
    std::vector<LeafSel> sel;
    std::vector<cf> full;                      // leaf store
    rqc_plan_info_t info{};
    // searched trees, best estimated time first (for timing on the device)
    struct Candidate {
        Tree tree;
        std::vector<int> sliced;
        double est;
    };
    std::vector<Candidate> candidates;
};

// Text table of the plan's launch program, one op per line.
std::string describe_program(const PlanCore &p);

// Contraction tree and sliced legs (user path/legs or the randomised search).
// With partial slicing (lc non-null, no user path or legs), the searched
// slicing starts with k0 near-input vertices (near_input_select on the best
// tree of a first search), and the tree is searched again on the network with
// those vertices projected; the memory slicing then adds legs to them.
void plan_tree(PlanCore &p, const int32_t *path, int32_t n_path_pairs, const std::vector<int> *user_sliced,
               const LightCones *lc = nullptr);
// k0 of Alg. 1: ceil(3 - log2 f), or opts.partial_k when set.
int partial_k0(const rqc_plan_opts &o);
// Appendix B, Alg. 1: S by SlicedVertexSelect, R from `norms` (which contracts
// the doubled network), X and F.
void plan_partial(PlanCore &p, const Network &net,
                  const std::function<std::vector<double>(const NetSpec &, const std::vector<int> &)> &norms);
// Batched/looped split, projections, leaf selection, lowering and plan info.
void plan_finish(PlanCore &p);

} // namespace rqc
