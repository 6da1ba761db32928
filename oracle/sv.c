/*
 * ORACLE -- test infrastructure only.  Plain FP64 state-vector simulator of the
 * circuit text format: |psi> = C|0^n>, applied gate by gate (Sec. I, where the
 * state psi = C|0> is defined).  Slow and obviously correct; it shares no code
 * with the HIP library.  Only tests, the smoke check and the bench's CPU
 * baseline call it.
 *
 * Conventions (stated once, used everywhere):
 *   - amplitude index x, bit q of x = value of qubit q;
 *   - single-qubit gates G_P = (I - iP)/sqrt(2), P in {X, Y, W}, W = (X+Y)/sqrt(2);
 *   - fSim(theta, phi) in the basis |b_a b_b> (b_a = bit of the first listed
 *     qubit, the high bit of the 2x2 block index):
 *       [[1,0,0,0],[0,cos t,-i sin t,0],[0,-i sin t,cos t,0],[0,0,0,e^{-i phi}]];
 *   - variables (tensor legs, the paper's "vertices", Appendix B): ids 0..n-1 are
 *     the inputs of the qubits; then, walking the gate lines in order, every
 *     single-qubit gate creates one new variable (its output), an fSim with
 *     theta = pi/2 creates none (it is a SWAP times a diagonal), and any other
 *     two-qubit gate creates two (first for qa, then for qb).
 *   - projecting variable v onto value b means zeroing the amplitudes whose bit
 *     on the qubit that carries v differs from b, right after v is created
 *     (for an input variable: before the first gate).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

enum { G_SX = 0, G_SY = 1, G_SW = 2, G_FSIM = 3 };

typedef struct {
    int kind;
    int qa, qb;
    double theta, phi; /* radians */
    int tnum, tden;    /* theta / pi as a fraction */
} gate_t;

typedef struct {
    int n;
    int n_gates;
    gate_t *gates;
} circ_t;

static int parse_frac(const char *s, int *num, int *den) {
    if (sscanf(s, "%d/%d", num, den) == 2 && *den != 0) return 0;
    if (sscanf(s, "%d", num) == 1) { *den = 1; return 0; }
    return -1;
}

/* Returns 0 on success, negative on a malformed line. */
static int parse(const char *text, circ_t *c) {
    c->n = -1;
    c->n_gates = 0;
    int cap = 1024;
    c->gates = (gate_t *)malloc(sizeof(gate_t) * cap);
    const char *p = text;
    char line[512];
    while (*p) {
        size_t len = strcspn(p, "\n");
        size_t cp = len < sizeof(line) - 1 ? len : sizeof(line) - 1;
        memcpy(line, p, cp);
        line[cp] = 0;
        p += len;
        if (*p == '\n') p++;
        char *hash = strchr(line, '#');
        if (hash) *hash = 0;
        char w0[64] = {0};
        if (sscanf(line, "%63s", w0) != 1) continue;
        if (!strcmp(w0, "qubits")) {
            if (sscanf(line, "%*s %d", &c->n) != 1) return -1;
        } else if (!strcmp(w0, "sx") || !strcmp(w0, "sy") || !strcmp(w0, "sw")) {
            int cyc, q;
            if (sscanf(line, "%*s %d %d", &cyc, &q) != 2) return -2;
            if (c->n_gates == cap) { cap *= 2; c->gates = (gate_t *)realloc(c->gates, sizeof(gate_t) * cap); }
            gate_t *g = &c->gates[c->n_gates++];
            memset(g, 0, sizeof(*g));
            g->kind = w0[1] == 'x' ? G_SX : (w0[1] == 'y' ? G_SY : G_SW);
            g->qa = q;
            g->qb = -1;
        } else if (!strcmp(w0, "fsim")) {
            int cyc, a, b;
            char ts[64], ps[64];
            if (sscanf(line, "%*s %d %d %d %63s %63s", &cyc, &a, &b, ts, ps) != 5) return -3;
            int tn, td, pn, pd;
            if (parse_frac(ts, &tn, &td) || parse_frac(ps, &pn, &pd)) return -4;
            if (c->n_gates == cap) { cap *= 2; c->gates = (gate_t *)realloc(c->gates, sizeof(gate_t) * cap); }
            gate_t *g = &c->gates[c->n_gates++];
            g->kind = G_FSIM;
            g->qa = a;
            g->qb = b;
            g->tnum = tn;
            g->tden = td;
            g->theta = M_PI * (double)tn / (double)td;
            g->phi = M_PI * (double)pn / (double)pd;
        }
        /* header lines grid/removed/cycles/rqc-circuit carry no gate */
    }
    if (c->n <= 0 || c->n > 40) return -5;
    for (int i = 0; i < c->n_gates; i++) {
        gate_t *g = &c->gates[i];
        if (g->qa < 0 || g->qa >= c->n) return -6;
        if (g->kind == G_FSIM && (g->qb < 0 || g->qb >= c->n || g->qb == g->qa)) return -6;
    }
    return 0;
}

static void one_qubit_matrix(int kind, cplx u[2][2]) {
    /* P in {X, Y, W}; G = (I - iP)/sqrt(2) */
    cplx P[2][2];
    const double r = 1.0 / sqrt(2.0);
    if (kind == G_SX) { P[0][0] = 0; P[0][1] = 1; P[1][0] = 1; P[1][1] = 0; }
    else if (kind == G_SY) { P[0][0] = 0; P[0][1] = -I; P[1][0] = I; P[1][1] = 0; }
    else { /* W = (X + Y)/sqrt(2) */
        P[0][0] = 0; P[0][1] = r * (1.0 - I); P[1][0] = r * (1.0 + I); P[1][1] = 0;
    }
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            u[a][b] = r * ((a == b ? 1.0 : 0.0) - I * P[a][b]);
}

static void fsim_matrix(double theta, double phi, cplx u[4][4]) {
    memset(u, 0, sizeof(cplx) * 16);
    u[0][0] = 1;
    u[1][1] = cos(theta);
    u[1][2] = -I * sin(theta);
    u[2][1] = -I * sin(theta);
    u[2][2] = cos(theta);
    u[3][3] = cexp(-I * phi);
}

static void apply_1q(cplx *s, int n, int q, cplx u[2][2]) {
    const int64_t half = (int64_t)1 << (n - 1);
    const int64_t lo = ((int64_t)1 << q) - 1;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < half; t++) {
        int64_t i0 = ((t & ~lo) << 1) | (t & lo);
        int64_t i1 = i0 | ((int64_t)1 << q);
        cplx a0 = s[i0], a1 = s[i1];
        s[i0] = u[0][0] * a0 + u[0][1] * a1;
        s[i1] = u[1][0] * a0 + u[1][1] * a1;
    }
}

static int64_t insert_zero(int64_t t, int q) {
    int64_t lo = ((int64_t)1 << q) - 1;
    return ((t & ~lo) << 1) | (t & lo);
}

static void apply_2q(cplx *s, int n, int qa, int qb, cplx u[4][4]) {
    const int64_t quarter = (int64_t)1 << (n - 2);
    const int lo = qa < qb ? qa : qb, hi = qa < qb ? qb : qa;
#pragma omp parallel for schedule(static)
    for (int64_t t = 0; t < quarter; t++) {
        int64_t base = insert_zero(insert_zero(t, lo), hi);
        int64_t idx[4];
        cplx in[4];
        for (int k = 0; k < 4; k++) {
            int ba = (k >> 1) & 1, bb = k & 1;
            idx[k] = base | ((int64_t)ba << qa) | ((int64_t)bb << qb);
            in[k] = s[idx[k]];
        }
        for (int r = 0; r < 4; r++) {
            cplx acc = 0;
            for (int k = 0; k < 4; k++) acc += u[r][k] * in[k];
            s[idx[r]] = acc;
        }
    }
}

static void project(cplx *s, int n, int q, int val) {
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; x++)
        if ((int)((x >> q) & 1) != val) s[x] = 0;
}

/* Number of qubits declared by the text, or a negative parse error. */
int rqco_num_qubits(const char *text) {
    circ_t c;
    int rc = parse(text, &c);
    int n = c.n;
    free(c.gates);
    return rc ? rc : n;
}

/* Number of gate lines, or a negative parse error. */
int rqco_num_gates(const char *text) {
    circ_t c;
    int rc = parse(text, &c);
    int g = c.n_gates;
    free(c.gates);
    return rc ? rc : g;
}

/*
 * Simulate the first `max_gates` gate lines (all if negative) on |0^n>.
 * `state` holds 2^n complex128 values (interleaved re, im) and is overwritten.
 * Each (proj_var[t], proj_val[t]) projects a variable as described above.
 * `nthreads` > 0 sets the OpenMP thread count.  Returns 0 or a negative error.
 */
int rqco_simulate(const char *text, int max_gates, int n_proj, const int *proj_var,
                  const int *proj_val, double *state, int nthreads) {
    circ_t c;
    int rc = parse(text, &c);
    if (rc) { free(c.gates); return rc; }
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    const int n = c.n;
    cplx *s = (cplx *)state;
    const int64_t N = (int64_t)1 << n;
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < N; x++) s[x] = 0;
    s[0] = 1;
    /* input variables */
    for (int t = 0; t < n_proj; t++)
        if (proj_var[t] >= 0 && proj_var[t] < n) project(s, n, proj_var[t], proj_val[t]);
    int next_var = n;
    int ng = max_gates < 0 || max_gates > c.n_gates ? c.n_gates : max_gates;
    for (int i = 0; i < ng; i++) {
        gate_t *g = &c.gates[i];
        int created[2] = {-1, -1}, created_q[2] = {-1, -1}, nc = 0;
        if (g->kind == G_FSIM) {
            cplx u[4][4];
            fsim_matrix(g->theta, g->phi, u);
            apply_2q(s, n, g->qa, g->qb, u);
            int swap_like = (g->tden != 0 && 2 * g->tnum == g->tden); /* theta = pi/2 */
            if (!swap_like) {
                created[nc] = next_var++; created_q[nc++] = g->qa;
                created[nc] = next_var++; created_q[nc++] = g->qb;
            }
        } else {
            cplx u[2][2];
            one_qubit_matrix(g->kind, u);
            apply_1q(s, n, g->qa, u);
            created[nc] = next_var++; created_q[nc++] = g->qa;
        }
        for (int k = 0; k < nc; k++)
            for (int t = 0; t < n_proj; t++)
                if (proj_var[t] == created[k]) project(s, n, created_q[k], proj_val[t]);
    }
    free(c.gates);
    return 0;
}

/* Amplitudes <x|C|0> for a list of indices, from an already simulated state. */
void rqco_gather(const double *state, const int64_t *idx, int64_t count, double *out) {
    for (int64_t t = 0; t < count; t++) {
        out[2 * t] = state[2 * idx[t]];
        out[2 * t + 1] = state[2 * idx[t] + 1];
    }
}

int rqco_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
