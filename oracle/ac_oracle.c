/*
 * ac_oracle.c -- serial Aho-Corasick oracle.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the bench's CPU-baseline leg may
 * load this library.  It shares no code, header, table or helper with the GPU
 * library and includes nothing from it.
 *
 * What it computes (paper, Section II): all occurrences of any of a finite set
 * of keywords in a text, found by a pattern matching machine built from the
 * keywords and driven over the text in a single pass.  The machine has the
 * three functions the paper names:
 *
 *   Goto     g(s, a): the keyword trie.  State 0 is the root; at the root every
 *            byte without an edge loops back to the root, so g(0, .) is total.
 *   Failure  f(s): the state to continue from when g(s, a) is undefined -- the
 *            state of the longest proper suffix of s's string that is also a
 *            keyword prefix (Fig. 4 draws these links).
 *   Output   out(s): every keyword recognised on entering s.  It is the set of
 *            keywords equal to s's string united with out(f(s)); that union is
 *            what reports the sub-patterns the paper says PFAC leaves out.
 *
 * Matching reads the text byte by byte (Fig. 3, "C"); each keyword p reported
 * at text position i (the index of its last byte) is an occurrence that starts
 * at i - |k_p| + 1.  Results are returned sorted by (start offset, keyword id).
 *
 * Keyword ids are input indices.  Bytes are raw unsigned 0..255, compared
 * exactly.  Duplicate keywords are allowed (each id is reported); an empty
 * keyword is rejected.
 *
 * Nothing here is tuned: children are kept in sorted arrays and searched by
 * bisection; only the root's total transition row is stored densely.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint8_t label;
    int32_t child;
} edge_t;

typedef struct {
    edge_t *edge;      /* children, sorted by label */
    int32_t n_edge, cap_edge;
    int32_t fail;
    int32_t *out;      /* Output function: keyword ids */
    int32_t n_out, cap_out;
} state_t;

typedef struct {
    state_t *st;
    int32_t n_states, cap_states;
    int32_t n_keywords;
    int64_t *len;          /* keyword lengths */
    int32_t root_row[256]; /* g(0, a), total */
} oracle_t;

typedef struct {
    int64_t *off;
    int32_t *pid;
    int64_t n, cap;
} result_t;

static int grow(void **p, int64_t *cap, int64_t need, size_t elem) {
    if (need <= *cap) return 0;
    int64_t nc = *cap ? *cap : 4;
    while (nc < need) nc *= 2;
    void *q = realloc(*p, (size_t)nc * elem);
    if (!q) return -1;
    *p = q;
    *cap = nc;
    return 0;
}

/* Goto lookup by bisection over the sorted children.  -1 = undefined. */
static int32_t child_of(const state_t *s, uint8_t a) {
    int32_t lo = 0, hi = s->n_edge;
    while (lo < hi) {
        int32_t mid = (lo + hi) / 2;
        if (s->edge[mid].label < a) lo = mid + 1;
        else hi = mid;
    }
    if (lo < s->n_edge && s->edge[lo].label == a) return s->edge[lo].child;
    return -1;
}

static int32_t new_state(oracle_t *m) {
    int64_t cap = m->cap_states;
    if (grow((void **)&m->st, &cap, (int64_t)m->n_states + 1, sizeof(state_t))) return -1;
    m->cap_states = (int32_t)cap;
    state_t *s = &m->st[m->n_states];
    memset(s, 0, sizeof(*s));
    return m->n_states++;
}

static int add_edge(oracle_t *m, int32_t from, uint8_t a, int32_t to) {
    state_t *s = &m->st[from];
    int64_t cap = s->cap_edge;
    if (grow((void **)&s->edge, &cap, (int64_t)s->n_edge + 1, sizeof(edge_t))) return -1;
    s->cap_edge = (int32_t)cap;
    int32_t pos = s->n_edge;
    while (pos > 0 && s->edge[pos - 1].label > a) {
        s->edge[pos] = s->edge[pos - 1];
        pos--;
    }
    s->edge[pos].label = a;
    s->edge[pos].child = to;
    s->n_edge++;
    return 0;
}

static int add_out(state_t *s, int32_t pid) {
    int64_t cap = s->cap_out;
    if (grow((void **)&s->out, &cap, (int64_t)s->n_out + 1, sizeof(int32_t))) return -1;
    s->cap_out = (int32_t)cap;
    s->out[s->n_out++] = pid;
    return 0;
}

/* Total Goto: undefined transitions of the root loop back to the root. */
static int32_t go(const oracle_t *m, int32_t s, uint8_t a) {
    if (s == 0) return m->root_row[a];
    return child_of(&m->st[s], a);
}

void oracle_free(oracle_t *m);

/*
 * Build the machine from n keywords packed as bytes[offs[i] .. offs[i+1]).
 * Returns NULL if a keyword is empty or memory runs out.
 */
oracle_t *oracle_build(const uint8_t *bytes, const int64_t *offs, int32_t n) {
    if (n < 0) return NULL;
    oracle_t *m = (oracle_t *)calloc(1, sizeof(oracle_t));
    if (!m) return NULL;
    m->n_keywords = n;
    m->len = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    if (!m->len || new_state(m) != 0) goto fail;

    /* Goto function: insert every keyword into the trie. */
    for (int32_t p = 0; p < n; ++p) {
        int64_t L = offs[p + 1] - offs[p];
        if (L <= 0) goto fail;
        m->len[p] = L;
        int32_t s = 0;
        for (int64_t j = 0; j < L; ++j) {
            uint8_t a = bytes[offs[p] + j];
            int32_t t = child_of(&m->st[s], a);
            if (t < 0) {
                t = new_state(m);
                if (t < 0 || add_edge(m, s, a, t)) goto fail;
            }
            s = t;
        }
        if (add_out(&m->st[s], p)) goto fail;
    }
    for (int a = 0; a < 256; ++a) {
        int32_t t = child_of(&m->st[0], (uint8_t)a);
        m->root_row[a] = t < 0 ? 0 : t;
    }

    /* Failure function, breadth first from the root. */
    {
        int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)m->n_states);
        if (!queue) goto fail;
        int64_t head = 0, tail = 0;
        state_t *root = &m->st[0];
        for (int32_t e = 0; e < root->n_edge; ++e) {
            int32_t s = root->edge[e].child;
            m->st[s].fail = 0;
            queue[tail++] = s;
        }
        while (head < tail) {
            int32_t r = queue[head++];
            for (int32_t e = 0; e < m->st[r].n_edge; ++e) {
                uint8_t a = m->st[r].edge[e].label;
                int32_t s = m->st[r].edge[e].child;
                queue[tail++] = s;
                int32_t st = m->st[r].fail;
                while (go(m, st, a) < 0) st = m->st[st].fail;
                int32_t f = go(m, st, a);
                m->st[s].fail = f;
                /* Output function: out(s) gains out(f(s)). */
                for (int32_t k = 0; k < m->st[f].n_out; ++k) {
                    if (add_out(&m->st[s], m->st[f].out[k])) {
                        free(queue);
                        goto fail;
                    }
                }
            }
        }
        free(queue);
    }
    return m;
fail:
    oracle_free(m);
    return NULL;
}

void oracle_free(oracle_t *m) {
    if (!m) return;
    for (int32_t i = 0; i < m->n_states; ++i) {
        free(m->st[i].edge);
        free(m->st[i].out);
    }
    free(m->st);
    free(m->len);
    free(m);
}

int32_t oracle_num_states(const oracle_t *m) { return m->n_states; }
int32_t oracle_goto(const oracle_t *m, int32_t s, int32_t a) { return go(m, s, (uint8_t)a); }
int32_t oracle_fail(const oracle_t *m, int32_t s) { return m->st[s].fail; }
int32_t oracle_out_count(const oracle_t *m, int32_t s) { return m->st[s].n_out; }
int32_t oracle_out_at(const oracle_t *m, int32_t s, int32_t k) { return m->st[s].out[k]; }

static int cmp_match(const void *x, const void *y) {
    const int64_t *a = (const int64_t *)x, *b = (const int64_t *)y;
    if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
    if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
    return 0;
}

/*
 * Scan text[0 .. n) once.  Returns NULL only if memory runs out.
 */
result_t *oracle_match(const oracle_t *m, const uint8_t *text, int64_t n) {
    result_t *r = (result_t *)calloc(1, sizeof(result_t));
    if (!r) return NULL;
    int64_t *pairs = NULL; /* (start, pid) pairs before sorting */
    int64_t cap = 0, cnt = 0;
    int32_t st = 0;
    for (int64_t i = 0; i < n; ++i) {
        uint8_t a = text[i];
        while (go(m, st, a) < 0) st = m->st[st].fail;
        st = go(m, st, a);
        const state_t *s = &m->st[st];
        for (int32_t k = 0; k < s->n_out; ++k) {
            int32_t p = s->out[k];
            if (grow((void **)&pairs, &cap, 2 * (cnt + 1), sizeof(int64_t))) goto fail;
            pairs[2 * cnt] = i - m->len[p] + 1;
            pairs[2 * cnt + 1] = p;
            cnt++;
        }
    }
    if (cnt) qsort(pairs, (size_t)cnt, 2 * sizeof(int64_t), cmp_match);
    r->n = cnt;
    r->off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cnt ? cnt : 1));
    r->pid = (int32_t *)malloc(sizeof(int32_t) * (size_t)(cnt ? cnt : 1));
    if (!r->off || !r->pid) goto fail;
    for (int64_t k = 0; k < cnt; ++k) {
        r->off[k] = pairs[2 * k];
        r->pid[k] = (int32_t)pairs[2 * k + 1];
    }
    free(pairs);
    return r;
fail:
    free(pairs);
    free(r->off);
    free(r->pid);
    free(r);
    return NULL;
}

int64_t oracle_result_count(const result_t *r) { return r->n; }

void oracle_result_copy(const result_t *r, int64_t *off, int32_t *pid) {
    if (r->n) {
        memcpy(off, r->off, sizeof(int64_t) * (size_t)r->n);
        memcpy(pid, r->pid, sizeof(int32_t) * (size_t)r->n);
    }
}

void oracle_result_free(result_t *r) {
    if (!r) return;
    free(r->off);
    free(r->pid);
    free(r);
}
