// Circuit text parser and hyper tensor-network builder.
//
// Each gate line becomes one leaf tensor.  A single-qubit gate U maps the
// wire's variable u to a new variable v: T[u, v] = U[v][u].  fSim(pi/2, phi)
// equals SWAP * diag(1, -i, -i, e^{-i phi}) (in the basis |b_a b_b>), so it
// becomes a two-leg diagonal tensor on the two current variables, which then
// trade wires; it creates no variable.  Any other two-qubit gate gives a
// four-leg tensor with two new variables.  Inputs are fixed to |0> (Sec. I:
// psi = C|0>) by restricting the first tensors that touch them.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>

#include "host.hpp"

namespace rqc {

static long gcdl(long a, long b) {
    a = std::labs(a);
    b = std::labs(b);
    while (b) {
        long t = a % b;
        a = b;
        b = t;
    }
    return a ? a : 1;
}

static bool parse_fraction(const char *s, long *num, long *den) {
    char *end = nullptr;
    long a = std::strtol(s, &end, 10);
    if (end == s) return false;
    long b = 1;
    if (*end == '/') {
        const char *p = end + 1;
        b = std::strtol(p, &end, 10);
        if (end == p || b == 0) return false;
    }
    if (*end != 0) return false;
    if (b < 0) {
        a = -a;
        b = -b;
    }
    long g = gcdl(a, b);
    *num = a / g;
    *den = b / g;
    return true;
}

Circuit parse_circuit(const char *text, size_t len) {
    Circuit c;
    c.n = -1;
    size_t pos = 0;
    int lineno = 0;
    std::string line;
    while (pos < len) {
        size_t e = pos;
        while (e < len && text[e] != '\n') e++;
        line.assign(text + pos, e - pos);
        pos = e + 1;
        lineno++;
        size_t h = line.find('#');
        if (h != std::string::npos) line.resize(h);
        char w[8][64];
        int nw = std::sscanf(line.c_str(), "%63s %63s %63s %63s %63s %63s %63s %63s", w[0], w[1], w[2],
                             w[3], w[4], w[5], w[6], w[7]);
        if (nw <= 0) continue;
        auto bad = [&](const char *why) {
            fail(RQC_EPARSE, "line " + std::to_string(lineno) + ": " + why);
        };
        auto toint = [&](const char *s) {
            char *end = nullptr;
            long v = std::strtol(s, &end, 10);
            if (end == s || *end != 0) bad("expected an integer");
            return (int)v;
        };
        std::string k = w[0];
        if (k == "qubits") {
            if (nw < 2) bad("qubits needs a count");
            c.n = toint(w[1]);
            if (c.n < 1 || c.n > 64) bad("qubit count must be 1..64");
        } else if (k == "sx" || k == "sy" || k == "sw") {
            if (nw < 3) bad("single-qubit gate needs <cycle> <qubit>");
            Gate g;
            g.kind = k == "sx" ? G_SX : (k == "sy" ? G_SY : G_SW);
            g.q[0] = toint(w[2]);
            c.gates.push_back(g);
        } else if (k == "fsim") {
            if (nw < 6) bad("fsim needs <cycle> <qa> <qb> <theta/pi> <phi/pi>");
            Gate g;
            g.kind = G_FSIM;
            g.q[0] = toint(w[2]);
            g.q[1] = toint(w[3]);
            if (!parse_fraction(w[4], &g.tnum, &g.tden) || !parse_fraction(w[5], &g.pnum, &g.pden))
                bad("angles must be fractions a/b");
            c.gates.push_back(g);
        } else if (k == "grid" || k == "removed" || k == "cycles" || k == "rqc-circuit") {
            // descriptive header lines
        } else {
            bad(("unknown statement '" + k + "'").c_str());
        }
    }
    if (c.n < 1) fail(RQC_EPARSE, "circuit declares no qubits");
    for (size_t i = 0; i < c.gates.size(); i++) {
        const Gate &g = c.gates[i];
        int nq = g.kind == G_FSIM ? 2 : 1;
        for (int j = 0; j < nq; j++)
            if (g.q[j] < 0 || g.q[j] >= c.n)
                fail(RQC_EPARSE, "gate " + std::to_string(i) + ": qubit out of range");
        if (nq == 2 && g.q[0] == g.q[1]) fail(RQC_EPARSE, "gate " + std::to_string(i) + ": repeated qubit");
    }
    return c;
}

// sqrt(P) = (I - iP)/sqrt(2)
static void one_qubit_matrix(int kind, cd u[2][2]) {
    const double r = 1.0 / std::sqrt(2.0);
    const cd I(0, 1);
    cd P[2][2];
    if (kind == G_SX) {
        P[0][0] = 0; P[0][1] = 1; P[1][0] = 1; P[1][1] = 0;
    } else if (kind == G_SY) {
        P[0][0] = 0; P[0][1] = -I; P[1][0] = I; P[1][1] = 0;
    } else {
        P[0][0] = 0; P[0][1] = r * (1.0 - I); P[1][0] = r * (1.0 + I); P[1][1] = 0;
    }
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++) u[a][b] = r * ((a == b ? 1.0 : 0.0) - I * P[a][b]);
}

static void fsim_matrix(const Gate &g, cd u[4][4]) {
    const double th = M_PI * (double)g.tnum / (double)g.tden;
    const double ph = M_PI * (double)g.pnum / (double)g.pden;
    const cd I(0, 1);
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) u[i][j] = 0;
    u[0][0] = 1;
    u[1][1] = u[2][2] = std::cos(th);
    u[1][2] = u[2][1] = -I * std::sin(th);
    u[3][3] = std::exp(-I * ph);
}

// Fix the legs that are input variables (ids < n) to value 0.
static void fix_inputs(Leaf &L, int n) {
    std::vector<int> keep;
    for (size_t i = 0; i < L.legs.size(); i++)
        if (L.legs[i] >= n) keep.push_back((int)i);
    if (keep.size() == L.legs.size()) return;
    std::vector<int> nl;
    for (int i : keep) nl.push_back(L.legs[i]);
    std::vector<cf> nd((size_t)1 << nl.size());
    for (size_t x = 0; x < nd.size(); x++) {
        size_t src = 0;
        for (size_t j = 0; j < keep.size(); j++)
            if ((x >> j) & 1) src |= (size_t)1 << keep[j];
        nd[x] = L.data[src];
    }
    L.legs = nl;
    L.data = nd;
}

Network build_network(const Circuit &c) {
    Network net;
    const int n = c.n;
    net.n_qubits = n;
    std::vector<int> cur(n);
    std::iota(cur.begin(), cur.end(), 0);
    int next = n;
    net.var_gate.assign(n, -1);
    for (size_t gi = 0; gi < c.gates.size(); gi++) {
        const Gate &g = c.gates[gi];
        Leaf L;
        if (g.kind != G_FSIM) {
            cd u[2][2];
            one_qubit_matrix(g.kind, u);
            int a = cur[g.q[0]], v = next++;
            net.var_gate.push_back((int)gi);
            net.gate_inputs.push_back({a});
            L.legs = {a, v};
            L.data.resize(4);
            // Stored as lambda * U with every entry exact in FP32, so rounding the
            // leaves leaves no systematic norm bias; 1/lambda is applied in FP64.
            // sqrt(X), sqrt(Y): entries are (1/sqrt 2) * {1, -1, -i}: lambda =
            // fl32(1/sqrt 2) * sqrt 2.  sqrt(W): diagonal 1/sqrt 2, off-diagonal
            // (+-1 +- i)/2; with o = 9093512 / 2^24 and d = 12860168 / 2^24
            // (d / o = 12860168 / 9093512, a convergent of sqrt 2 scaled by 8,
            // exact to 3e-14), lambda = 2 o.
            double lam;
            if (g.kind == G_SW) lam = 2.0 * (9093512.0 / 16777216.0);
            else lam = (double)(float)(1.0 / std::sqrt(2.0)) * std::sqrt(2.0);
            for (int x = 0; x < 4; x++) {
                cd e = lam * u[(x >> 1) & 1][x & 1];
                L.data[x] = cf((float)e.real(), (float)e.imag());
            }
            if (g.kind == G_SW) {
                const float d = 12860168.0f / 16777216.0f;
                L.data[0] = cf(d, 0.f);
                L.data[3] = cf(d, 0.f);
            }
            L.scale = lam;
            cur[g.q[0]] = v;
        } else if (g.swap_like()) {
            const double ph = M_PI * (double)g.pnum / (double)g.pden;
            int a = cur[g.q[0]], b = cur[g.q[1]];
            net.gate_inputs.push_back({a, b});
            L.legs = {a, b};
            // e^{-i phi} as the complex64 value of least |.|^2 - 1 within a few
            // ulps of the rounded phase, so repeated use adds no norm drift
            float bc = (float)std::cos(ph), bs = (float)-std::sin(ph);
            double best = 1e300;
            const float c0 = bc, s0 = bs;
            for (int i = -4; i <= 4; i++)
                for (int j = -4; j <= 4; j++) {
                    float c = c0, s = s0;
                    for (int t = 0; t < std::abs(i); t++) c = std::nextafter(c, i > 0 ? 2.f : -2.f);
                    for (int t = 0; t < std::abs(j); t++) s = std::nextafter(s, j > 0 ? 2.f : -2.f);
                    double err = std::fabs((double)c * c + (double)s * s - 1.0) +
                                 std::fabs(std::atan2((double)s, (double)c) + ph) * 0.5;
                    if (err < best) best = err, bc = c, bs = s;
                }
            L.data = {cf(1, 0), cf(0, -1), cf(0, -1), cf(bc, bs)};
            std::swap(cur[g.q[0]], cur[g.q[1]]);
        } else {
            cd u[4][4];
            fsim_matrix(g, u);
            int a = cur[g.q[0]], b = cur[g.q[1]];
            int a2 = next++, b2 = next++;
            net.var_gate.push_back((int)gi);
            net.var_gate.push_back((int)gi);
            net.gate_inputs.push_back({a, b});
            L.legs = {a, b, a2, b2};
            L.data.resize(16);
            for (int x = 0; x < 16; x++) {
                int ia = x & 1, ib = (x >> 1) & 1, oa = (x >> 2) & 1, ob = (x >> 3) & 1;
                L.data[x] = cf(u[2 * oa + ob][2 * ia + ib]);
            }
            cur[g.q[0]] = a2;
            cur[g.q[1]] = b2;
        }
        net.leaves.push_back(std::move(L));
    }
    net.n_vars = next;
    net.out_var = cur;
    for (int q = 0; q < n; q++)
        if (cur[q] < n)
            fail(RQC_EINVAL, "qubit " + std::to_string(q) +
                                 " ends on an input variable (no single-qubit gate on its wire)");
    for (auto &L : net.leaves) fix_inputs(L, n);
    // legs of a leaf are kept in creation order; sort them for a canonical layout
    for (auto &L : net.leaves) {
        std::vector<int> order(L.legs.size());
        std::iota(order.begin(), order.end(), 0);
        std::sort(order.begin(), order.end(), [&](int i, int j) { return L.legs[i] < L.legs[j]; });
        bool sorted = true;
        for (size_t i = 0; i < order.size(); i++) sorted &= order[i] == (int)i;
        if (sorted) continue;
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
    return net;
}

} // namespace rqc
