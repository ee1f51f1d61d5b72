/*
 * Plain CPU oracle for exact simulation (ES) of an AIG miter.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this.  It shares no code with the
 * GPU path and is deliberately slow and direct.
 *
 * What it computes (paper, Section 2.1 and Section 2.2 "Exact Simulation"):
 * the circuit is a latch-free AIG; a miter is equivalent iff its output is 0
 * for every primary-input assignment; exact simulation enumerates all 2^n
 * assignments and checks the miter output.  A multi-output file is read as a
 * miter whose output is the OR of all outputs (the OR step of the miter
 * construction).  Pattern p assigns bit i of p to the i-th primary input in
 * file order.  The answer is the lowest failing p, or "none".
 *
 * Algorithm, one pattern at a time:
 *   1. read the ASCII AIGER file with the reader below;
 *   2. order the AND gates topologically (file order when it already is one);
 *   3. for each p: set the inputs from the bits of p, evaluate every AND gate
 *      in order as (a ^ ca) & (b ^ cb), OR the output literals;
 *   4. split [lo, hi) into contiguous chunks, one per thread; each thread
 *      scans its chunk in ascending order, stops at its first failure or once
 *      p reaches the best failure found so far; the result is the minimum.
 *
 * Parity pins for this file live in the test suite: closed-form products and
 * sums of products, minterm circuits with known unique failures, and small
 * hand-worked miters.
 */
#include "es_oracle.h"

#include <pthread.h>
#include <stdatomic.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

struct oracle_aig {
    uint32_t maxvar;
    uint32_t num_inputs;
    uint32_t num_outputs;
    uint32_t num_ands;
    uint32_t *input_var;   /* [num_inputs] variable of the i-th input */
    uint32_t *out_lit;     /* [num_outputs] */
    uint32_t *and_var;     /* [num_ands] in topological order */
    uint32_t *and_r0;      /* [num_ands] */
    uint32_t *and_r1;      /* [num_ands] */
};

/* ------------------------------------------------------------------------ */
/* ASCII AIGER reader                                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    const char *s;
    size_t n, i;
} cursor;

static int skip_spaces(cursor *c) {
    while (c->i < c->n && c->s[c->i] == ' ') c->i++;
    return c->i < c->n;
}

static int read_uint(cursor *c, uint64_t *v) {
    skip_spaces(c);
    if (c->i >= c->n || c->s[c->i] < '0' || c->s[c->i] > '9') return 0;
    uint64_t x = 0;
    while (c->i < c->n && c->s[c->i] >= '0' && c->s[c->i] <= '9') {
        x = x * 10 + (uint64_t)(c->s[c->i] - '0');
        if (x > 0xFFFFFFFFull) return 0;
        c->i++;
    }
    *v = x;
    return 1;
}

static int end_line(cursor *c) {
    skip_spaces(c);
    if (c->i < c->n && c->s[c->i] == '\r') c->i++;
    if (c->i >= c->n) return 1;
    if (c->s[c->i] != '\n') return 0;
    c->i++;
    return 1;
}

static void set_err(char *err, size_t errlen, const char *msg) {
    if (err && errlen) {
        strncpy(err, msg, errlen - 1);
        err[errlen - 1] = 0;
    }
}

void oracle_free(oracle_aig *g) {
    if (!g) return;
    free(g->input_var);
    free(g->out_lit);
    free(g->and_var);
    free(g->and_r0);
    free(g->and_r1);
    free(g);
}

int oracle_parse_aag(const char *text, size_t len, oracle_aig **out, char *err, size_t errlen) {
    cursor c = {text, len, 0};
    uint64_t M, I, L, O, A;
    *out = NULL;
    if (len < 4 || memcmp(text, "aag", 3) != 0 || text[3] != ' ') {
        set_err(err, errlen, "not an ASCII AIGER file (header 'aag')");
        return ORACLE_ERR_PARSE;
    }
    c.i = 3;
    if (!read_uint(&c, &M) || !read_uint(&c, &I) || !read_uint(&c, &L) || !read_uint(&c, &O) ||
        !read_uint(&c, &A)) {
        set_err(err, errlen, "bad header");
        return ORACLE_ERR_PARSE;
    }
    /* AIGER 1.9 optional counts: bad states, constraints, justice, fairness. */
    for (int k = 0; k < 4; ++k) {
        uint64_t extra;
        size_t save = c.i;
        if (!read_uint(&c, &extra)) { c.i = save; break; }
        if (extra != 0) {
            set_err(err, errlen, "bad-state/constraint/justice/fairness sections are not combinational");
            return ORACLE_ERR_UNSUPPORTED;
        }
    }
    if (!end_line(&c)) { set_err(err, errlen, "bad header line"); return ORACLE_ERR_PARSE; }
    if (L != 0) { set_err(err, errlen, "latches are not supported (combinational AIGs only)"); return ORACLE_ERR_UNSUPPORTED; }
    if (M < I + A) { set_err(err, errlen, "header: M < I + A"); return ORACLE_ERR_PARSE; }
    if (I > 64) { set_err(err, errlen, "more than 64 inputs"); return ORACLE_ERR_UNSUPPORTED; }

    oracle_aig *g = (oracle_aig *)calloc(1, sizeof(*g));
    g->maxvar = (uint32_t)M;
    g->num_inputs = (uint32_t)I;
    g->num_outputs = (uint32_t)O;
    g->num_ands = (uint32_t)A;
    g->input_var = (uint32_t *)calloc(I ? I : 1, sizeof(uint32_t));
    g->out_lit = (uint32_t *)calloc(O ? O : 1, sizeof(uint32_t));
    uint32_t *lhs = (uint32_t *)calloc(A ? A : 1, sizeof(uint32_t));
    uint32_t *r0 = (uint32_t *)calloc(A ? A : 1, sizeof(uint32_t));
    uint32_t *r1 = (uint32_t *)calloc(A ? A : 1, sizeof(uint32_t));
    /* kind[v]: 0 undefined, 1 constant, 2 input, 3 and; gate[v]: index of its AND line */
    uint8_t *kind = (uint8_t *)calloc(M + 1, 1);
    uint32_t *gate = (uint32_t *)calloc(M + 1, sizeof(uint32_t));
    int rc = ORACLE_OK;
    kind[0] = 1;

    for (uint64_t k = 0; k < I && rc == ORACLE_OK; ++k) {
        uint64_t lit;
        if (!read_uint(&c, &lit) || !end_line(&c) || (lit & 1) || lit < 2 || (lit >> 1) > M ||
            kind[lit >> 1]) {
            set_err(err, errlen, "bad input line");
            rc = ORACLE_ERR_PARSE;
            break;
        }
        kind[lit >> 1] = 2;
        g->input_var[k] = (uint32_t)(lit >> 1);
    }
    for (uint64_t k = 0; k < O && rc == ORACLE_OK; ++k) {
        uint64_t lit;
        if (!read_uint(&c, &lit) || !end_line(&c) || (lit >> 1) > M) {
            set_err(err, errlen, "bad output line");
            rc = ORACLE_ERR_PARSE;
            break;
        }
        g->out_lit[k] = (uint32_t)lit;
    }
    for (uint64_t k = 0; k < A && rc == ORACLE_OK; ++k) {
        uint64_t l, a, b;
        if (!read_uint(&c, &l) || !read_uint(&c, &a) || !read_uint(&c, &b) || !end_line(&c) ||
            (l & 1) || l < 2 || (l >> 1) > M || (a >> 1) > M || (b >> 1) > M || kind[l >> 1]) {
            set_err(err, errlen, "bad AND line");
            rc = ORACLE_ERR_PARSE;
            break;
        }
        kind[l >> 1] = 3;
        gate[l >> 1] = (uint32_t)k;
        lhs[k] = (uint32_t)l;
        r0[k] = (uint32_t)a;
        r1[k] = (uint32_t)b;
    }
    /* every referenced variable must be defined */
    for (uint64_t k = 0; k < O && rc == ORACLE_OK; ++k)
        if (!kind[g->out_lit[k] >> 1]) { set_err(err, errlen, "output uses an undefined variable"); rc = ORACLE_ERR_PARSE; }
    for (uint64_t k = 0; k < A && rc == ORACLE_OK; ++k)
        if (!kind[r0[k] >> 1] || !kind[r1[k] >> 1]) { set_err(err, errlen, "AND uses an undefined variable"); rc = ORACLE_ERR_PARSE; }

    /* Topological order by depth-first search over fan-ins (iterative). */
    if (rc == ORACLE_OK) {
        g->and_var = (uint32_t *)malloc((A ? A : 1) * sizeof(uint32_t));
        g->and_r0 = (uint32_t *)malloc((A ? A : 1) * sizeof(uint32_t));
        g->and_r1 = (uint32_t *)malloc((A ? A : 1) * sizeof(uint32_t));
        uint8_t *state = (uint8_t *)calloc(A ? A : 1, 1); /* 0 new, 1 on stack, 2 done */
        uint32_t *stack = (uint32_t *)malloc((A ? A : 1) * sizeof(uint32_t));
        uint32_t emitted = 0;
        for (uint64_t root = 0; root < A && rc == ORACLE_OK; ++root) {
            if (state[root]) continue;
            uint32_t sp = 0;
            stack[sp++] = (uint32_t)root;
            state[root] = 1;
            while (sp && rc == ORACLE_OK) {
                uint32_t k = stack[sp - 1];
                uint32_t pending = UINT32_MAX;
                uint32_t fan[2] = {r0[k] >> 1, r1[k] >> 1};
                for (int f = 0; f < 2; ++f) {
                    if (kind[fan[f]] != 3) continue;
                    uint32_t j = gate[fan[f]];
                    if (state[j] == 1) { set_err(err, errlen, "combinational cycle"); rc = ORACLE_ERR_PARSE; }
                    else if (state[j] == 0) { pending = j; break; }
                }
                if (rc != ORACLE_OK) break;
                if (pending != UINT32_MAX) {
                    state[pending] = 1;
                    stack[sp++] = pending;
                } else {
                    state[k] = 2;
                    --sp;
                    g->and_var[emitted] = lhs[k] >> 1;
                    g->and_r0[emitted] = r0[k];
                    g->and_r1[emitted] = r1[k];
                    ++emitted;
                }
            }
        }
        free(state);
        free(stack);
    }
    free(lhs);
    free(r0);
    free(r1);
    free(kind);
    free(gate);
    if (rc != ORACLE_OK) {
        oracle_free(g);
        return rc;
    }
    *out = g;
    return ORACLE_OK;
}

uint32_t oracle_num_inputs(const oracle_aig *g) { return g->num_inputs; }
uint32_t oracle_num_outputs(const oracle_aig *g) { return g->num_outputs; }
uint32_t oracle_num_ands(const oracle_aig *g) { return g->num_ands; }

/* ------------------------------------------------------------------------ */
/* Evaluation of one pattern                                                 */
/* ------------------------------------------------------------------------ */

/* Evaluate every variable of g at pattern p into val[0..maxvar]. */
static void simulate(const oracle_aig *g, uint64_t p, uint8_t *val) {
    val[0] = 0;
    for (uint32_t i = 0; i < g->num_inputs; ++i) val[g->input_var[i]] = (uint8_t)((p >> i) & 1u);
    for (uint32_t k = 0; k < g->num_ands; ++k) {
        uint32_t a = g->and_r0[k], b = g->and_r1[k];
        uint8_t va = (uint8_t)(val[a >> 1] ^ (a & 1u));
        uint8_t vb = (uint8_t)(val[b >> 1] ^ (b & 1u));
        val[g->and_var[k]] = (uint8_t)(va & vb);
    }
}

static uint8_t literal_value(const uint8_t *val, uint32_t lit) { return (uint8_t)(val[lit >> 1] ^ (lit & 1u)); }

static int miter_value(const oracle_aig *g, const uint8_t *val) {
    int m = 0;
    for (uint32_t j = 0; j < g->num_outputs; ++j) m |= literal_value(val, g->out_lit[j]);
    return m;
}

int oracle_eval_outputs(const oracle_aig *g, const uint64_t *ps, size_t k, uint64_t *out_words) {
    if (g->num_outputs > 64) return ORACLE_ERR_UNSUPPORTED;
    uint8_t *val = (uint8_t *)malloc(g->maxvar + 1);
    for (size_t t = 0; t < k; ++t) {
        simulate(g, ps[t], val);
        uint64_t w = 0;
        for (uint32_t j = 0; j < g->num_outputs; ++j) w |= (uint64_t)literal_value(val, g->out_lit[j]) << j;
        out_words[t] = w;
    }
    free(val);
    return ORACLE_OK;
}

int oracle_eval_miter(const oracle_aig *g, const uint64_t *ps, size_t k, uint8_t *out) {
    uint8_t *val = (uint8_t *)malloc(g->maxvar + 1);
    for (size_t t = 0; t < k; ++t) {
        simulate(g, ps[t], val);
        out[t] = (uint8_t)miter_value(g, val);
    }
    free(val);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ */
/* Exhaustive scan for the lowest failing pattern                            */
/* ------------------------------------------------------------------------ */

typedef struct {
    const oracle_aig *g;
    uint64_t lo, hi;
    _Atomic uint64_t *best;
    uint64_t evaluated;
} scan_job;

static void *scan_worker(void *arg) {
    scan_job *job = (scan_job *)arg;
    uint8_t *val = (uint8_t *)malloc(job->g->maxvar + 1);
    uint64_t count = 0;
    for (uint64_t p = job->lo; p < job->hi; ++p) {
        if ((count & 1023u) == 0 && p >= atomic_load_explicit(job->best, memory_order_relaxed)) break;
        simulate(job->g, p, val);
        ++count;
        if (miter_value(job->g, val)) {
            uint64_t cur = atomic_load(job->best);
            while (p < cur && !atomic_compare_exchange_weak(job->best, &cur, p)) {
            }
            break;
        }
    }
    job->evaluated = count;
    free(val);
    return NULL;
}

uint64_t oracle_lowest_failure(const oracle_aig *g, uint64_t lo, uint64_t hi, int threads,
                               uint64_t *evaluated) {
    _Atomic uint64_t best = ORACLE_NONE;
    if (threads < 1) threads = 1;
    if (hi <= lo) {
        if (evaluated) *evaluated = 0;
        return ORACLE_NONE;
    }
    uint64_t span = hi - lo;
    if ((uint64_t)threads > span) threads = (int)span;
    scan_job *jobs = (scan_job *)calloc((size_t)threads, sizeof(scan_job));
    pthread_t *tid = (pthread_t *)calloc((size_t)threads, sizeof(pthread_t));
    uint64_t chunk = span / (uint64_t)threads, extra = span % (uint64_t)threads, start = lo;
    for (int t = 0; t < threads; ++t) {
        uint64_t len = chunk + ((uint64_t)t < extra ? 1 : 0);
        jobs[t].g = g;
        jobs[t].lo = start;
        jobs[t].hi = start + len;
        jobs[t].best = &best;
        start += len;
    }
    for (int t = 1; t < threads; ++t) pthread_create(&tid[t], NULL, scan_worker, &jobs[t]);
    scan_worker(&jobs[0]);
    uint64_t total = jobs[0].evaluated;
    for (int t = 1; t < threads; ++t) {
        pthread_join(tid[t], NULL);
        total += jobs[t].evaluated;
    }
    free(jobs);
    free(tid);
    if (evaluated) *evaluated = total;
    return atomic_load(&best);
}
