/*
 * oracle/zs_oracle.c - TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU implementation of the ZSMILES codec
 * (Accordi et al., "ZSMILES: an approach for efficient SMILES storage for
 * random access in Virtual Screening").  It exists to check the GPU library
 * and to be timed beside it.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the product never does.  It
 * shares no code, header or table with the GPU path.
 *
 * Every function cites the passage of the paper it follows.  Where the paper
 * is silent the reading taken is stated at the function (the list of readings
 * is kept with the design notes):
 *   - the escape space precedes its literal (Sec. IV-D-2 decoder);
 *   - an escape edge of cost 2 exists at every position (Sec. IV-D-1);
 *   - among minimum-length parses the one whose sequence of consumed lengths
 *     is lexicographically greatest is emitted ("T1");
 *   - ring IDs are assigned at each ring's closing label as the smallest ID
 *     not used by a ring that closed inside it ("mex at close", Sec. IV-A);
 *   - malformed ring syntax, or an ID >= 100, leaves the line unchanged.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ZO_OK 0
#define ZO_EINVAL (-1)
#define ZO_ENOSPC (-2)
#define ZO_ECORRUPT (-3)

#define ZO_F_PREPROCESS 1u
#define ZO_LMAX_CAP 16

typedef struct {
    uint8_t len[256];              /* 0 = byte is not a code                */
    uint8_t exp[256][ZO_LMAX_CAP]; /* expansion of each code               */
    int ncodes;
    int lmax;
    uint8_t sorted[256];           /* codes sorted by expansion, for lookup */
} zo_dict;

/* ------------------------------------------------------------------------ */
/* Dictionary                                                                */
/* ------------------------------------------------------------------------ */

static int is_code_byte(int b) { return (b >= 0x21 && b <= 0x7E) || (b >= 0xA1 && b <= 0xFF); }

static const zo_dict *g_sort_dict;
static int cmp_exp(const uint8_t *a, int la, const uint8_t *b, int lb) {
    int l = la < lb ? la : lb;
    int c = memcmp(a, b, (size_t)l);
    if (c) return c;
    return la - lb;
}
static int cmp_codes(const void *pa, const void *pb) {
    int a = *(const uint8_t *)pa, b = *(const uint8_t *)pb;
    return cmp_exp(g_sort_dict->exp[a], g_sort_dict->len[a], g_sort_dict->exp[b], g_sort_dict->len[b]);
}

/*
 * Build a dictionary from a code table (Sec. IV-B/IV-C: one fixed table that
 * maps a printable byte to a pattern).  Returns ZO_EINVAL when a code byte is
 * not printable (space is the escape, newline the separator), an expansion is
 * empty, longer than 16 bytes or holds a byte outside 0x21..0x7E, or two codes
 * share an expansion.
 */
int zo_dict_init(zo_dict *d, const uint8_t *len, const uint8_t *exp /* [256][16] */) {
    memset(d, 0, sizeof *d);
    for (int b = 0; b < 256; b++) {
        int L = len[b];
        if (L == 0) continue;
        if (!is_code_byte(b) || L > ZO_LMAX_CAP) return ZO_EINVAL;
        for (int j = 0; j < L; j++) {
            int c = exp[b * ZO_LMAX_CAP + j];
            if (c < 0x21 || c > 0x7E) return ZO_EINVAL;
        }
        d->len[b] = (uint8_t)L;
        memcpy(d->exp[b], exp + b * ZO_LMAX_CAP, (size_t)L);
        d->sorted[d->ncodes++] = (uint8_t)b;
        if (L > d->lmax) d->lmax = L;
    }
    g_sort_dict = d;
    qsort(d->sorted, (size_t)d->ncodes, 1, cmp_codes);
    for (int i = 1; i < d->ncodes; i++) {
        int a = d->sorted[i - 1], b = d->sorted[i];
        if (cmp_exp(d->exp[a], d->len[a], d->exp[b], d->len[b]) == 0) return ZO_EINVAL;
    }
    return ZO_OK;
}

/* The code whose expansion is exactly s[0..L), or -1 (binary search). */
static int lookup(const zo_dict *d, const uint8_t *s, int L) {
    int lo = 0, hi = d->ncodes - 1;
    while (lo <= hi) {
        int mid = (lo + hi) / 2;
        int b = d->sorted[mid];
        int c = cmp_exp(d->exp[b], d->len[b], s, L);
        if (c == 0) return b;
        if (c < 0) lo = mid + 1;
        else hi = mid - 1;
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* Pre-processing: ring-ID reuse (Sec. IV-A)                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t pos;   /* position of the label token in the line   */
    int toklen;    /* 1 for a digit, 3 for %nn                   */
    int value;     /* label value 0..99                          */
    int ring;      /* ring the label belongs to                  */
} zo_label;

static int is_digit(int c) { return c >= '0' && c <= '9'; }

/*
 * Rewrite the ring-closure labels of one SMILES line so that ring IDs are
 * reused (Sec. IV-A).  Labels are a digit, or '%' and two digits, outside
 * square brackets (digits inside brackets are isotopes, charges or hydrogen
 * counts; Sec. II).  The first label of a value opens a ring, the next label
 * of the same value closes it.  Rings are numbered in the order of their
 * closing labels: ring R, opened at o and closed at c, gets the smallest
 * non-negative ID not held by any ring whose closing label lies strictly
 * between o and c.  A ring enclosing another therefore gets a larger ID than
 * the inner one (the innermost choice of Sec. IV-A), disjoint rings reuse 0,
 * and the paper's Dibenzoylmethane example is reproduced.  IDs 0..9 are
 * written as one digit, 10..99 as '%' and two digits.  Bond symbols before a
 * label stay where they are.  A line with unbalanced brackets, a '%' not
 * followed by two digits, an unclosed ring, or needing an ID >= 100 is copied
 * unchanged.  Writes y (capacity >= 3*n) and returns its length.
 */
int64_t zo_preprocess(const uint8_t *x, int64_t n, uint8_t *y) {
    zo_label *lab = (zo_label *)malloc(sizeof(zo_label) * (size_t)(n + 1));
    int nl = 0, inbr = 0, bad = 0;
    for (int64_t i = 0; i < n && !bad; i++) {
        int c = x[i];
        if (c == '[') {
            if (inbr) bad = 1;
            inbr = 1;
        } else if (c == ']') {
            if (!inbr) bad = 1;
            inbr = 0;
        } else if (!inbr && is_digit(c)) {
            lab[nl].pos = i; lab[nl].toklen = 1; lab[nl].value = c - '0'; nl++;
        } else if (!inbr && c == '%') {
            if (i + 2 < n && is_digit(x[i + 1]) && is_digit(x[i + 2])) {
                lab[nl].pos = i; lab[nl].toklen = 3;
                lab[nl].value = (x[i + 1] - '0') * 10 + (x[i + 2] - '0');
                nl++;
                i += 2;
            } else {
                bad = 1;
            }
        }
    }
    if (inbr) bad = 1;

    /* pair labels into rings: open_of[v] is the open label of value v */
    int open_of[100];
    for (int v = 0; v < 100; v++) open_of[v] = -1;
    int nr = 0;
    int *ring_open = (int *)malloc(sizeof(int) * (size_t)(nl / 2 + 1));
    int *ring_close = (int *)malloc(sizeof(int) * (size_t)(nl / 2 + 1));
    for (int j = 0; j < nl && !bad; j++) {
        int v = lab[j].value;
        if (open_of[v] < 0) {
            open_of[v] = j;
        } else {
            ring_open[nr] = open_of[v];
            ring_close[nr] = j;
            lab[open_of[v]].ring = nr;
            lab[j].ring = nr;
            nr++;
            open_of[v] = -1;
        }
    }
    for (int v = 0; v < 100 && !bad; v++)
        if (open_of[v] >= 0) bad = 1;

    /* rings are listed in closing order; assign IDs by the mex rule */
    int *id = (int *)malloc(sizeof(int) * (size_t)(nr + 1));
    for (int r = 0; r < nr && !bad; r++) {
        unsigned char used[101];
        memset(used, 0, sizeof used);
        for (int q = 0; q < r; q++) {
            /* ring q closed before ring r; does its closing label lie inside r? */
            if (ring_close[q] > ring_open[r] && ring_close[q] < ring_close[r]) {
                if (id[q] <= 100) used[id[q]] = 1;
            }
        }
        int v = 0;
        while (v <= 100 && used[v]) v++;
        id[r] = v;
        if (v >= 100) bad = 1;
    }

    int64_t m = 0;
    if (bad) {
        memcpy(y, x, (size_t)n);
        m = n;
    } else {
        int j = 0;
        for (int64_t i = 0; i < n;) {
            if (j < nl && lab[j].pos == i) {
                int v = id[lab[j].ring];
                if (v < 10) {
                    y[m++] = (uint8_t)('0' + v);
                } else {
                    y[m++] = '%';
                    y[m++] = (uint8_t)('0' + v / 10);
                    y[m++] = (uint8_t)('0' + v % 10);
                }
                i += lab[j].toklen;
                j++;
            } else {
                y[m++] = x[i++];
            }
        }
    }
    free(lab);
    free(ring_open);
    free(ring_close);
    free(id);
    return m;
}

/* ------------------------------------------------------------------------ */
/* Post-processing after decompression (Sec. IV-D: "optionally               */
/* post-processed"; the paper gives no definition, the one below is ours)    */
/* ------------------------------------------------------------------------ */

/*
 * Relabel the ring closures of one decompressed line the way SMILES writers
 * usually number them: reading left to right, a ring's opening label takes
 * the smallest label >= 1 that no ring open at that point holds, and its
 * closing label repeats it.  Labels 1..9 are one digit, 10..99 '%' and two
 * digits.  Tokens, pairing and malformed lines as in zo_preprocess (labels
 * are digits or '%nn' outside brackets; the first label of a value opens a
 * ring, the next closes it); a malformed line, or one that would need a label
 * above 99, is copied unchanged.  Writes y (capacity >= 3*n) and returns its
 * length.
 */
int64_t zo_postprocess(const uint8_t *x, int64_t n, uint8_t *y) {
    /* label tokens: position, token length, value */
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    int *tlen = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    int *val = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    int *newl = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    int nt = 0, inbr = 0, bad = 0;
    for (int64_t i = 0; i < n && !bad; i++) {
        int c = x[i];
        if (c == '[') {
            if (inbr) bad = 1;
            inbr = 1;
        } else if (c == ']') {
            if (!inbr) bad = 1;
            inbr = 0;
        } else if (!inbr && is_digit(c)) {
            pos[nt] = i; tlen[nt] = 1; val[nt] = c - '0'; nt++;
        } else if (!inbr && c == '%') {
            if (i + 2 < n && is_digit(x[i + 1]) && is_digit(x[i + 2])) {
                pos[nt] = i; tlen[nt] = 3; val[nt] = (x[i + 1] - '0') * 10 + (x[i + 2] - '0'); nt++;
                i += 2;
            } else {
                bad = 1;
            }
        }
    }
    if (inbr) bad = 1;
    /* walk the tokens in order: an opening takes the smallest free label >= 1,
       the closing of the same value gives it back */
    int open_tok[100], held[101];
    for (int v = 0; v < 100; v++) open_tok[v] = -1;
    for (int v = 0; v <= 100; v++) held[v] = 0;
    for (int j = 0; j < nt && !bad; j++) {
        int v = val[j];
        if (open_tok[v] < 0) {
            int l = 1;
            while (l < 100 && held[l]) l++;
            if (l >= 100) {
                bad = 1;
                break;
            }
            held[l] = 1;
            newl[j] = l;
            open_tok[v] = j;
        } else {
            int l = newl[open_tok[v]];
            newl[j] = l;
            held[l] = 0;
            open_tok[v] = -1;
        }
    }
    for (int v = 0; v < 100 && !bad; v++)
        if (open_tok[v] >= 0) bad = 1;
    int64_t m = 0;
    if (bad) {
        memcpy(y, x, (size_t)n);
        m = n;
    } else {
        int j = 0;
        for (int64_t i = 0; i < n;) {
            if (j < nt && pos[j] == i) {
                int l = newl[j];
                if (l < 10) {
                    y[m++] = (uint8_t)('0' + l);
                } else {
                    y[m++] = '%';
                    y[m++] = (uint8_t)('0' + l / 10);
                    y[m++] = (uint8_t)('0' + l % 10);
                }
                i += tlen[j];
                j++;
            } else {
                y[m++] = x[i++];
            }
        }
    }
    free(pos);
    free(tlen);
    free(val);
    free(newl);
    return m;
}

/* ------------------------------------------------------------------------ */
/* Compression of one line (Sec. IV-D-1)                                     */
/* ------------------------------------------------------------------------ */

/*
 * Shortest path over the graph of Sec. IV-D-1: nodes are the positions
 * 0..m of the (pre-processed) line s, an edge i -> i+L of cost 1 exists for
 * every dictionary pattern s[i..i+L), and an escape edge i -> i+1 of cost 2
 * (a space followed by the literal byte) exists at every position.  The graph
 * is acyclic with positive weights, so the backward recurrence
 *     cost[m] = 0,
 *     cost[i] = min(2 + cost[i+1], min over patterns L at i of 1 + cost[i+L])
 * gives the same costs as Dijkstra.  The path is then walked from the
 * beginning, printing one output token per edge; at each node the longest
 * optimal edge is taken (reading "T1").  Writes the compressed line (no
 * newline) to y, capacity >= 2*m, and returns its length, equal to cost[0].
 */
int64_t zo_compress_pre(const zo_dict *d, const uint8_t *s, int64_t m, uint8_t *y) {
    int64_t *cost = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    cost[m] = 0;
    for (int64_t i = m - 1; i >= 0; i--) {
        int64_t best = 2 + cost[i + 1];
        for (int L = 1; L <= d->lmax && i + L <= m; L++) {
            if (lookup(d, s + i, L) >= 0 && 1 + cost[i + L] < best) best = 1 + cost[i + L];
        }
        cost[i] = best;
    }
    int64_t o = 0;
    for (int64_t i = 0; i < m;) {
        int take = 0, code = -1;
        for (int L = d->lmax; L >= 1; L--) {
            if (i + L > m) continue;
            int b = lookup(d, s + i, L);
            if (b >= 0 && 1 + cost[i + L] == cost[i]) {
                take = L;
                code = b;
                break;
            }
        }
        if (take) {
            y[o++] = (uint8_t)code;
            i += take;
        } else {
            y[o++] = ' ';
            y[o++] = s[i];
            i += 1;
        }
    }
    free(cost);
    return o;
}

/* Input bytes of a SMILES line are printable ASCII, space included (Sec. II). */
static int line_ok(const uint8_t *x, int64_t n) {
    for (int64_t i = 0; i < n; i++)
        if (x[i] < 0x20 || x[i] > 0x7E) return 0;
    return 1;
}

/* Compress one raw line: optional pre-processing, then the parse above. */
int64_t zo_compress_line(const zo_dict *d, const uint8_t *x, int64_t n, uint32_t flags, uint8_t *y) {
    if (!(flags & ZO_F_PREPROCESS)) return zo_compress_pre(d, x, n, y);
    uint8_t *p = (uint8_t *)malloc((size_t)(3 * n + 1));
    int64_t m = zo_preprocess(x, n, p);
    int64_t o = zo_compress_pre(d, p, m, y);
    free(p);
    return o;
}

/* ------------------------------------------------------------------------ */
/* Decompression of one line (Sec. IV-D-2)                                   */
/* ------------------------------------------------------------------------ */

/*
 * Table lookup per byte: a code prints its expansion; a space means the next
 * byte is printed as it is.  A space with no byte after it, a byte that is
 * not a code, or an escaped byte outside 0x20..0x7E (the compressor only
 * escapes bytes of a SMILES line, so such a literal cannot come from it, and
 * a newline there would break the line framing) is corrupt input.  Writes y
 * (capacity >= lmax*n) and returns the length, or -1 when corrupt.
 */
int64_t zo_decompress_line(const zo_dict *d, const uint8_t *c, int64_t n, uint8_t *y) {
    int64_t o = 0;
    for (int64_t j = 0; j < n;) {
        if (c[j] == ' ') {
            if (j + 1 >= n) return -1;
            if (c[j + 1] < 0x20 || c[j + 1] > 0x7E) return -1;
            y[o++] = c[j + 1];
            j += 2;
        } else {
            int L = d->len[c[j]];
            if (L == 0) return -1;
            memcpy(y + o, d->exp[c[j]], (size_t)L);
            o += L;
            j += 1;
        }
    }
    return o;
}

/* ------------------------------------------------------------------------ */
/* Buffers: one SMILES per line, line k in = line k out (Sec. I)             */
/* ------------------------------------------------------------------------ */

/*
 * Line k of a buffer is in[off[k] .. off[k+1]-1) and in[off[k+1]-1] is its
 * newline; the last line may instead end at a virtual newline one past the
 * buffer (off[n] = in_bytes + 1).  Returns 1 when line k is framed this way.
 */
static int frame_ok(const uint8_t *in, uint64_t in_bytes, const uint64_t *off, uint64_t n, uint64_t k) {
    uint64_t a = off[k], b = off[k + 1];
    if (b <= a || b > in_bytes + 1) return 0;
    if (b == in_bytes + 1) return k + 1 == n;
    return in[b - 1] == '\n';
}

static void note_bad(int64_t *first_bad, int *code, int64_t k, int c) {
    if (*first_bad < 0 || k < *first_bad) {
        *first_bad = k;
        *code = c;
    }
}

/*
 * Compress every line of a buffer, in order.  out_off[0] = 0 and
 * out_off[k+1] = out_off[k] + (compressed length of line k) + 1.  A line that
 * is badly framed (EINVAL) or holds a byte outside 0x20..0x7E (ECORRUPT)
 * yields an empty output line; the result code is that of the first bad line
 * and *first_bad its index.  With out == NULL only out_off is computed.  If
 * the output does not fit out_cap the code is ENOSPC (when no line is bad) and
 * out holds nothing useful.
 */
int zo_compress(const zo_dict *d, const uint8_t *in, uint64_t in_bytes, const uint64_t *in_off,
                uint64_t n, uint32_t flags, uint8_t *out, uint64_t out_cap, uint64_t *out_off,
                int64_t *first_bad) {
    int code = ZO_OK;
    *first_bad = -1;
    out_off[0] = 0;
    uint8_t *tmp = NULL;
    int64_t tmp_cap = 0;
    for (uint64_t k = 0; k < n; k++) {
        int64_t len = 0;
        if (!frame_ok(in, in_bytes, in_off, n, k)) {
            note_bad(first_bad, &code, (int64_t)k, ZO_EINVAL);
        } else {
            const uint8_t *x = in + in_off[k];
            int64_t xl = (int64_t)(in_off[k + 1] - in_off[k] - 1);
            if (!line_ok(x, xl)) {
                note_bad(first_bad, &code, (int64_t)k, ZO_ECORRUPT);
            } else {
                if (6 * xl + 1 > tmp_cap) {
                    free(tmp);
                    tmp_cap = 6 * xl + 64;
                    tmp = (uint8_t *)malloc((size_t)tmp_cap);
                }
                len = zo_compress_line(d, x, xl, flags, tmp);
            }
        }
        uint64_t o = out_off[k];
        out_off[k + 1] = o + (uint64_t)len + 1;
        if (out && out_off[k + 1] <= out_cap) {
            memcpy(out + o, tmp, (size_t)len);
            out[o + (uint64_t)len] = '\n';
        }
    }
    free(tmp);
    if (code == ZO_OK && out && out_off[n] > out_cap) code = ZO_ENOSPC;
    return code;
}

static int64_t decompress_one(const zo_dict *d, const uint8_t *in, uint64_t in_bytes, const uint64_t *in_off,
                              uint64_t n, uint64_t k, uint8_t **tmp, int64_t *tmp_cap, int *err) {
    if (!frame_ok(in, in_bytes, in_off, n, k)) {
        *err = ZO_EINVAL;
        return 0;
    }
    int64_t cl = (int64_t)(in_off[k + 1] - in_off[k] - 1);
    int64_t need = cl * (d->lmax > 1 ? d->lmax : 1) + 1;
    if (need > *tmp_cap) {
        free(*tmp);
        *tmp_cap = need + 64;
        *tmp = (uint8_t *)malloc((size_t)*tmp_cap);
    }
    int64_t len = zo_decompress_line(d, in + in_off[k], cl, *tmp);
    if (len < 0) {
        *err = ZO_ECORRUPT;
        return 0;
    }
    *err = ZO_OK;
    return len;
}

/* Decompress every line of a buffer (Sec. IV-D-2); conventions as zo_compress. */
int zo_decompress(const zo_dict *d, const uint8_t *in, uint64_t in_bytes, const uint64_t *in_off,
                  uint64_t n, uint8_t *out, uint64_t out_cap, uint64_t *out_off, int64_t *first_bad) {
    int code = ZO_OK;
    *first_bad = -1;
    out_off[0] = 0;
    uint8_t *tmp = NULL;
    int64_t tmp_cap = 0;
    for (uint64_t k = 0; k < n; k++) {
        int err;
        int64_t len = decompress_one(d, in, in_bytes, in_off, n, k, &tmp, &tmp_cap, &err);
        if (err) note_bad(first_bad, &code, (int64_t)k, err);
        uint64_t o = out_off[k];
        out_off[k + 1] = o + (uint64_t)len + 1;
        if (out && out_off[k + 1] <= out_cap) {
            if (len) memcpy(out + o, tmp, (size_t)len);
            out[o + (uint64_t)len] = '\n';
        }
    }
    free(tmp);
    if (code == ZO_OK && out && out_off[n] > out_cap) code = ZO_ENOSPC;
    return code;
}

/*
 * Random access (Sec. I: separable lines, so any line can be read alone):
 * decompress lines ids[0..n_ids) and pack them in request order.  An id not
 * below n gives EINVAL for that request; *first_bad is a request index.
 */
int zo_decompress_lines(const zo_dict *d, const uint8_t *in, uint64_t in_bytes, const uint64_t *in_off,
                        uint64_t n, const uint64_t *ids, uint64_t n_ids, uint8_t *out, uint64_t out_cap,
                        uint64_t *out_off, int64_t *first_bad) {
    int code = ZO_OK;
    *first_bad = -1;
    out_off[0] = 0;
    uint8_t *tmp = NULL;
    int64_t tmp_cap = 0;
    for (uint64_t r = 0; r < n_ids; r++) {
        int err = ZO_OK;
        int64_t len = 0;
        if (ids[r] >= n) err = ZO_EINVAL;
        else len = decompress_one(d, in, in_bytes, in_off, n, ids[r], &tmp, &tmp_cap, &err);
        if (err) note_bad(first_bad, &code, (int64_t)r, err);
        uint64_t o = out_off[r];
        out_off[r + 1] = o + (uint64_t)len + 1;
        if (out && out_off[r + 1] <= out_cap) {
            if (len) memcpy(out + o, tmp, (size_t)len);
            out[o + (uint64_t)len] = '\n';
        }
    }
    free(tmp);
    if (code == ZO_OK && out && out_off[n_ids] > out_cap) code = ZO_ENOSPC;
    return code;
}

/*
 * Line index of a newline-separated buffer (one SMILES per line, Sec. I):
 * off[0] = 0 and off[k+1] is one past the k-th newline; an unterminated last
 * line ends at a virtual newline, off[n] = len + 1.  Returns the number of
 * lines; when off_cap < lines + 1 nothing beyond off_cap is written and the
 * return value is still the line count.
 */
int64_t zo_index_lines(const uint8_t *buf, uint64_t len, uint64_t *off, uint64_t off_cap) {
    int64_t k = 0;
    if (off_cap > 0) off[0] = 0;
    for (uint64_t p = 0; p < len; p++) {
        if (buf[p] == '\n') {
            k++;
            if ((uint64_t)k < off_cap) off[k] = p + 1;
        }
    }
    if (len > 0 && buf[len - 1] != '\n') {
        k++;
        if ((uint64_t)k < off_cap) off[k] = len + 1;
    }
    return k;
}

/*
 * Pre-process every line of a buffer (Sec. IV-A), keeping the framing:
 * out_off[k+1] = out_off[k] + (pre-processed length of line k) + 1.  Lines are
 * assumed well framed.  out must hold 3 * in_bytes + n bytes.
 */
void zo_preprocess_buffer(const uint8_t *in, const uint64_t *in_off, uint64_t n, uint8_t *out, uint64_t *out_off) {
    out_off[0] = 0;
    for (uint64_t k = 0; k < n; k++) {
        int64_t xl = (int64_t)(in_off[k + 1] - in_off[k] - 1);
        int64_t m = zo_preprocess(in + in_off[k], xl, out + out_off[k]);
        out[out_off[k] + (uint64_t)m] = '\n';
        out_off[k + 1] = out_off[k] + (uint64_t)m + 1;
    }
}

/* Post-process every line of a buffer (same framing rules as zo_preprocess_buffer). */
void zo_postprocess_buffer(const uint8_t *in, const uint64_t *in_off, uint64_t n, uint8_t *out, uint64_t *out_off) {
    out_off[0] = 0;
    for (uint64_t k = 0; k < n; k++) {
        int64_t xl = (int64_t)(in_off[k + 1] - in_off[k] - 1);
        int64_t m = zo_postprocess(in + in_off[k], xl, out + out_off[k]);
        out[out_off[k] + (uint64_t)m] = '\n';
        out_off[k + 1] = out_off[k] + (uint64_t)m + 1;
    }
}

/* Size helpers for callers of the library. */
uint64_t zo_sizeof_dict(void) { return sizeof(zo_dict); }
