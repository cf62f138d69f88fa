/*
 * oracle/train_dict.c - TEST INFRASTRUCTURE: dictionary generation, used to
 * produce the frozen dictionaries and as the reference of the trainer tests.
 * Not part of the GPU path.
 *
 * Algorithm 1 of the paper (Sec. IV-C) with the rank of Eq. (1):
 *   1. count every substring s of every training line with
 *      Lmin <= |s| <= Lmax (occurrences, overlapping ones included);
 *   2. repeat T times: take the substring of highest rank, add it to the
 *      dictionary, remove it from the candidates, update the other ranks.
 * rank_{p,t} = occ_p * (l_p - overlap_{p,t}).  The paper leaves update_rank
 * and "overlap with the patterns selected so far" open; the reading here is
 * overlap_{p,t} = the longest common substring of p with any pattern selected
 * before step t.  Ties go to the higher rank, then the longer pattern, then
 * the bytewise smaller one.  The loop stops early when no candidate has a
 * positive rank.  The training lines are pre-processed first when asked
 * (Sec. V-B: dictionaries are trained on pre-processed data).
 *
 * Patterns are at most 16 bytes (Sec. V-C sweeps Lmax up to 15).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int64_t zo_preprocess(const uint8_t *x, int64_t n, uint8_t *y);

#define ZO_TRAIN_LMAX 16

typedef struct {
    uint8_t b[ZO_TRAIN_LMAX]; /* the substring, zero padded */
    uint32_t len;             /* 0 = empty table entry */
    uint32_t occ;
} cand;

/* FNV-1a over the bytes and the length (any fixed hash will do: it only
   places entries in the table, it decides nothing). */
static uint64_t hash_sub(const uint8_t *s, int len) {
    uint64_t h = 1469598103934665603ull;
    for (int i = 0; i < len; i++) {
        h ^= s[i];
        h *= 1099511628211ull;
    }
    h ^= (uint64_t)len;
    h *= 1099511628211ull;
    return h ^ (h >> 29);
}

/* Longest common substring of a and b: the classic table of common suffix
   lengths, c[i][j] = c[i-1][j-1] + 1 when a[i-1] == b[j-1], else 0. */
static int lcs_len(const uint8_t *a, int la, const uint8_t *b, int lb) {
    int c[ZO_TRAIN_LMAX + 1][ZO_TRAIN_LMAX + 1];
    int best = 0;
    for (int i = 0; i <= la; i++) c[i][0] = 0;
    for (int j = 0; j <= lb; j++) c[0][j] = 0;
    for (int i = 1; i <= la; i++)
        for (int j = 1; j <= lb; j++) {
            c[i][j] = (a[i - 1] == b[j - 1]) ? c[i - 1][j - 1] + 1 : 0;
            if (c[i][j] > best) best = c[i][j];
        }
    return best;
}

/* Double the table and re-insert its entries. */
static int grow(cand **tab, uint64_t *cap) {
    uint64_t nc = 2 * *cap;
    cand *t = (cand *)calloc(nc, sizeof(cand));
    if (!t) return 0;
    for (uint64_t i = 0; i < *cap; i++) {
        const cand *e = &(*tab)[i];
        if (!e->len) continue;
        uint64_t h = hash_sub(e->b, (int)e->len) & (nc - 1);
        while (t[h].len) h = (h + 1) & (nc - 1);
        t[h] = *e;
    }
    free(*tab);
    *tab = t;
    *cap = nc;
    return 1;
}

/* key order of Eq. (1) with the tie-breaks: is (r1, p1) ahead of (r2, p2)? */
static int ahead(int64_t r1, const cand *p1, int64_t r2, const cand *p2) {
    if (r1 != r2) return r1 > r2;
    if (p1->len != p2->len) return p1->len > p2->len;
    return memcmp(p1->b, p2->b, p1->len) < 0;
}

/*
 * Train on lines buf[off[k] .. off[k+1]-1).  Writes up to T patterns into
 * pat[T][16] / pat_len[T] in selection order and returns how many were
 * chosen; -1 for bad parameters, -2 when out of memory.
 */
int zo_train_dict(const uint8_t *buf, const uint64_t *off, uint64_t n, int preprocess, int lmin, int lmax,
                  int T, uint8_t *pat, uint8_t *pat_len) {
    if (lmax > ZO_TRAIN_LMAX || lmin < 1 || lmin > lmax || T < 0) return -1;
    int64_t longest = 0;
    for (uint64_t k = 0; k < n; k++) {
        int64_t xl = (int64_t)(off[k + 1] - off[k] - 1);
        if (xl > longest) longest = xl;
    }
    /* open-addressing table, doubled whenever it is half full */
    uint64_t cap = 1u << 16;
    cand *tab = (cand *)calloc(cap, sizeof(cand));
    uint8_t *tmp = (uint8_t *)malloc((size_t)(3 * longest + 64));
    if (!tab || !tmp) {
        free(tab);
        free(tmp);
        return -2;
    }
    uint64_t used = 0;
    /* Algorithm 1, first loop: count the substrings */
    for (uint64_t k = 0; k < n; k++) {
        const uint8_t *x = buf + off[k];
        int64_t xl = (int64_t)(off[k + 1] - off[k] - 1);
        int64_t m;
        if (preprocess) {
            m = zo_preprocess(x, xl, tmp);
        } else {
            memcpy(tmp, x, (size_t)xl);
            m = xl;
        }
        for (int64_t i = 0; i < m; i++) {
            for (int L = lmin; L <= lmax && i + L <= m; L++) {
                const uint8_t *s = tmp + i;
                uint64_t h = hash_sub(s, L) & (cap - 1);
                while (tab[h].len && !(tab[h].len == (uint32_t)L && memcmp(tab[h].b, s, (size_t)L) == 0))
                    h = (h + 1) & (cap - 1);
                if (!tab[h].len) {
                    memcpy(tab[h].b, s, (size_t)L);
                    tab[h].len = (uint32_t)L;
                    used++;
                }
                tab[h].occ++;
                if (2 * used > cap && !grow(&tab, &cap)) {
                    free(tab);
                    free(tmp);
                    return -2;
                }
            }
        }
    }
    free(tmp);
    /* the candidates, compacted */
    cand *c = (cand *)malloc(sizeof(cand) * (used ? used : 1));
    int *overlap = (int *)calloc(used ? used : 1, sizeof(int));
    unsigned char *taken = (unsigned char *)calloc(used ? used : 1, 1);
    if (!c || !overlap || !taken) {
        free(tab);
        free(c);
        free(overlap);
        free(taken);
        return -2;
    }
    uint64_t nc = 0;
    for (uint64_t h = 0; h < cap; h++)
        if (tab[h].len) c[nc++] = tab[h];
    free(tab);
    /* Algorithm 1, second loop: T selections, each followed by the overlap update */
    int chosen = 0;
    for (int t = 0; t < T; t++) {
        int64_t best = -1;
        uint64_t bi = 0;
        for (uint64_t i = 0; i < nc; i++) {
            if (taken[i]) continue;
            int64_t r = (int64_t)c[i].occ * (int64_t)((int)c[i].len - overlap[i]);
            if (best < 0 || ahead(r, &c[i], best, &c[bi])) {
                best = r;
                bi = i;
            }
        }
        if (best <= 0) break;
        taken[bi] = 1;
        memcpy(pat + (size_t)ZO_TRAIN_LMAX * chosen, c[bi].b, ZO_TRAIN_LMAX);
        pat_len[chosen] = (uint8_t)c[bi].len;
        chosen++;
        for (uint64_t i = 0; i < nc; i++) {
            if (taken[i] || overlap[i] >= (int)c[i].len) continue;
            int l = lcs_len(c[i].b, (int)c[i].len, c[bi].b, (int)c[bi].len);
            if (l > overlap[i]) overlap[i] = l;
        }
    }
    free(c);
    free(overlap);
    free(taken);
    return chosen;
}
