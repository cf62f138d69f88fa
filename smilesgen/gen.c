/*
 * smilesgen/gen.c - seeded synthetic SMILES generator.
 *
 * Produces newline-separated, SMILES-like ASCII lines from a random
 * molecular-graph grammar: atoms C N O S F Cl Br, aromatic c n o s, bracket
 * atoms [NH+] [O-] (and [NH3+], which carries a digit inside brackets, when
 * asked for), branches '(' ')', bond symbols '=' '#', and ring-closure labels
 * 1-9 then %10-%99.  Ring labels are never reused inside one line (a fresh
 * label per ring, lowest free one once 99 is passed), which is how raw SMILES
 * writers number rings and what the ring-ID pre-processing of the paper
 * (Sec. IV-A) then compacts.
 *
 * The generator holds none of the codec's arithmetic: it only writes input
 * bytes.  Randomness is a per-line counter generator: line k of seed s draws
 * from SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014) started from a state derived from (s, k), so any
 * line can be produced alone, in parallel, and identically on every machine.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t dist;           /* 0: uniform integer length in [lo, hi]; 1: log-normal */
    int32_t lo, hi;         /* uniform range, or clip range of the log-normal      */
    double median, sigma;   /* log-normal: exp(N(ln median, sigma^2))              */
    double long_frac;       /* probability that a line is drawn in long mode       */
    int32_t long_lo, long_hi; /* long-mode length, uniform integer                 */
    int32_t bracket_digits; /* also emit [NH3+] (a digit inside brackets)          */
    int32_t reserved;
} smg_params;

/* SplitMix64 step: the published constants of the generator. */
static inline uint64_t sm_next(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static inline uint64_t line_state(uint64_t seed, uint64_t line) {
    uint64_t a = seed;
    uint64_t h = sm_next(&a);
    uint64_t b = h ^ (line * 0xD1B54A32D192ED03ull + 0x8CB92BA72F3D8DD7ull);
    sm_next(&b);
    return b;
}

static inline double unif(uint64_t *s) { return (double)(sm_next(s) >> 11) * (1.0 / 9007199254740992.0); }
static inline int irange(uint64_t *s, int lo, int hi) { return lo + (int)(sm_next(s) % (uint64_t)(hi - lo + 1)); }

static double normal(uint64_t *s) {
    double u1 = unif(s), u2 = unif(s);
    if (u1 < 1e-300) u1 = 1e-300;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* atom table: text and weight (normalised at use) */
static const char *ATOMS[] = {"C", "c", "O", "N", "n", "F", "Cl", "Br", "S", "o", "s", "[B]"};
static const double ATOM_W[] = {0.35, 0.25, 0.08, 0.07, 0.05, 0.03, 0.03, 0.02, 0.02, 0.01, 0.01, 0.05};
#define N_ATOMS 12

typedef struct {
    char *p;
    int n, cap;
} sbuf;

static inline void put(sbuf *b, const char *t) {
    while (*t && b->n < b->cap) b->p[b->n++] = *t++;
}
static inline void putc1(sbuf *b, char c) {
    if (b->n < b->cap) b->p[b->n++] = c;
}

static void put_label(sbuf *b, int v) {
    if (v < 10) {
        putc1(b, (char)('0' + v));
    } else {
        putc1(b, '%');
        putc1(b, (char)('0' + v / 10));
        putc1(b, (char)('0' + v % 10));
    }
}

static void put_atom(sbuf *b, uint64_t *s, int bracket_digits) {
    double u = unif(s) * 0.97; /* sum of ATOM_W */
    int a = 0;
    for (; a < N_ATOMS - 1; a++) {
        if (u < ATOM_W[a]) break;
        u -= ATOM_W[a];
    }
    if (a == N_ATOMS - 1) {
        int k = (int)(sm_next(s) % (bracket_digits ? 3u : 2u));
        put(b, k == 0 ? "[NH+]" : (k == 1 ? "[O-]" : "[NH3+]"));
    } else {
        put(b, ATOMS[a]);
    }
}

/* Generate one line (without '\n') into out[0..cap); returns its length. */
static int gen_line(const smg_params *P, uint64_t seed, uint64_t line, char *out, int cap) {
    uint64_t st = line_state(seed, line);
    uint64_t *s = &st;
    int longm = (P->long_frac > 0.0) && (unif(s) < P->long_frac);
    int target;
    if (longm) {
        target = irange(s, P->long_lo, P->long_hi);
    } else if (P->dist == 1) {
        double L = P->median * exp(P->sigma * normal(s));
        target = (int)floor(L + 0.5);
        if (target < P->lo) target = P->lo;
        if (target > P->hi) target = P->hi;
    } else {
        target = irange(s, P->lo, P->hi);
    }
    const int max_depth = longm ? 12 : 4;
    const double p_ring = longm ? 0.30 : 0.08;
    const int ring_lo = longm ? 15 : 4, ring_hi = longm ? 60 : 6;
    const double p_branch = longm ? 0.22 : 0.15;
    const double p_bclose = longm ? 0.20 : 0.30;

    sbuf b = {out, 0, cap};
    int open_label[100], close_at[100], n_open = 0;
    unsigned char in_use[100];
    memset(in_use, 0, sizeof in_use);
    int next_label = 1, atoms = 0, depth = 0, after_open = 1;
    int stop = target - 3;
    if (stop < 1) stop = 1;
    while (b.n < stop) {
        if (!after_open) {
            double u = unif(s);
            if (u < 0.10) putc1(&b, '=');
            else if (u < 0.12) putc1(&b, '#');
        }
        put_atom(&b, s, P->bracket_digits);
        atoms++;
        after_open = 0;
        /* close rings that are due at this atom */
        for (int r = 0; r < n_open;) {
            if (close_at[r] <= atoms) {
                put_label(&b, open_label[r]);
                in_use[open_label[r]] = 0;
                open_label[r] = open_label[n_open - 1];
                close_at[r] = close_at[n_open - 1];
                n_open--;
            } else {
                r++;
            }
        }
        /* maybe open a ring on this atom */
        if (unif(s) < p_ring && n_open < 99) {
            int v = -1;
            if (next_label <= 99) {
                v = next_label++;
            } else {
                for (int c = 1; c <= 99; c++)
                    if (!in_use[c]) { v = c; break; }
            }
            if (v > 0) {
                in_use[v] = 1;
                open_label[n_open] = v;
                close_at[n_open] = atoms + irange(s, ring_lo, ring_hi);
                n_open++;
                put_label(&b, v);
            }
        }
        /* branches */
        double u = unif(s);
        if (depth > 0 && u < p_bclose) {
            putc1(&b, ')');
            depth--;
        } else if (depth < max_depth && u < p_bclose + p_branch) {
            putc1(&b, '(');
            depth++;
            after_open = 1;
        }
    }
    /* finish: an atom to carry the closing labels, then close branches */
    if (after_open || (b.n > 0 && b.p[b.n - 1] == ')')) {
        put_atom(&b, s, P->bracket_digits);
    }
    for (int r = 0; r < n_open; r++) put_label(&b, open_label[r]);
    while (depth-- > 0) putc1(&b, ')');
    return b.n;
}

#define LINE_CAP 8192

/*
 * Generate lines [first, first+n) of `seed` into buf with offsets off[0..n]
 * (off[0] = 0, off[k+1] = off[k] + len_k + 1, each line ends in '\n').
 * buf may be NULL to only compute off.  Returns total bytes, or -1 if cap is
 * too small (then buf holds nothing useful).
 */
int64_t smg_generate(const smg_params *P, uint64_t seed, uint64_t first, uint64_t n,
                     uint8_t *buf, uint64_t cap, uint64_t *off, int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int32_t *lens = (int32_t *)malloc(sizeof(int32_t) * (n ? n : 1));
    if (!lens) return -1;
#pragma omp parallel
    {
        char *tmp = (char *)malloc(LINE_CAP);
#pragma omp for schedule(static, 4096)
        for (int64_t k = 0; k < (int64_t)n; k++) lens[k] = gen_line(P, seed, first + (uint64_t)k, tmp, LINE_CAP);
        free(tmp);
    }
    off[0] = 0;
    for (uint64_t k = 0; k < n; k++) off[k + 1] = off[k] + (uint64_t)lens[k] + 1;
    int64_t total = (int64_t)off[n];
    free(lens);
    if (!buf) return total;
    if ((uint64_t)total > cap) return -1;
#pragma omp parallel
    {
        char *tmp = (char *)malloc(LINE_CAP);
#pragma omp for schedule(static, 4096)
        for (int64_t k = 0; k < (int64_t)n; k++) {
            int L = gen_line(P, seed, first + (uint64_t)k, tmp, LINE_CAP);
            memcpy(buf + off[k], tmp, (size_t)L);
            buf[off[k] + (uint64_t)L] = '\n';
        }
        free(tmp);
    }
    return total;
}
