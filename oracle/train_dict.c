/*
 * oracle/train_dict.c - TEST INFRASTRUCTURE: dictionary generation used once to
 * produce the frozen default dictionary.  Not part of the GPU path.
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
 * the bytewise smaller one.  The training lines are pre-processed first when
 * asked (Sec. V-B: dictionaries are trained on pre-processed data).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int64_t zo_preprocess(const uint8_t *x, int64_t n, uint8_t *y);

typedef struct {
    uint64_t key; /* up to 8 bytes, little-endian packed */
    uint32_t len;
    uint32_t occ;
} cand;

static uint64_t hash64(uint64_t k, uint32_t l) {
    k ^= (uint64_t)l * 0x9E3779B97F4A7C15ull;
    k ^= k >> 33;
    k *= 0xFF51AFD7ED558CCDull;
    k ^= k >> 33;
    k *= 0xC4CEB9FE1A85EC53ull;
    return k ^ (k >> 33);
}

static int lcs_len(const uint8_t *a, int la, const uint8_t *b, int lb) {
    int best = 0;
    for (int i = 0; i < la; i++)
        for (int j = 0; j < lb; j++) {
            int k = 0;
            while (i + k < la && j + k < lb && a[i + k] == b[j + k]) k++;
            if (k > best) best = k;
        }
    return best;
}

static void unpack(uint64_t key, int len, uint8_t *out) {
    for (int i = 0; i < len; i++) out[i] = (uint8_t)(key >> (8 * i));
}

/*
 * Train on lines buf[off[k] .. off[k+1]-1).  Writes up to T patterns into
 * pat[T][8] / pat_len[T] in selection order and returns how many were chosen.
 * Lmax <= 8 (patterns are packed into 64-bit keys).
 */
int zo_train_dict(const uint8_t *buf, const uint64_t *off, uint64_t n, int preprocess, int lmin, int lmax,
                  int T, uint8_t *pat, uint8_t *pat_len) {
    if (lmax > 8 || lmin < 1 || lmin > lmax) return -1;
    uint64_t cap = 1u << 22;
    cand *tab = (cand *)calloc(cap, sizeof(cand));
    uint64_t used = 0;
    uint8_t *tmp = NULL;
    int64_t tmp_cap = 0;
    for (uint64_t k = 0; k < n; k++) {
        const uint8_t *x = buf + off[k];
        int64_t xl = (int64_t)(off[k + 1] - off[k] - 1);
        if (3 * xl + 1 > tmp_cap) {
            free(tmp);
            tmp_cap = 3 * xl + 64;
            tmp = (uint8_t *)malloc((size_t)tmp_cap);
        }
        int64_t m;
        if (preprocess) {
            m = zo_preprocess(x, xl, tmp);
        } else {
            memcpy(tmp, x, (size_t)xl);
            m = xl;
        }
        for (int64_t i = 0; i < m; i++) {
            uint64_t key = 0;
            for (int L = 1; L <= lmax && i + L <= m; L++) {
                key |= (uint64_t)tmp[i + L - 1] << (8 * (L - 1));
                if (L < lmin) continue;
                uint64_t h = hash64(key, (uint32_t)L) & (cap - 1);
                while (tab[h].len && !(tab[h].key == key && tab[h].len == (uint32_t)L)) h = (h + 1) & (cap - 1);
                if (!tab[h].len) {
                    tab[h].key = key;
                    tab[h].len = (uint32_t)L;
                    used++;
                    if (used * 2 > cap) { free(tab); free(tmp); return -2; }
                }
                tab[h].occ++;
            }
        }
    }
    free(tmp);
    /* compact the candidates */
    cand *c = (cand *)malloc(sizeof(cand) * (used ? used : 1));
    uint64_t nc = 0;
    for (uint64_t h = 0; h < cap; h++)
        if (tab[h].len) c[nc++] = tab[h];
    free(tab);
    int *overlap = (int *)calloc(nc ? nc : 1, sizeof(int));
    unsigned char *taken = (unsigned char *)calloc(nc ? nc : 1, 1);
    int chosen = 0;
    uint8_t a[8], b[8];
    for (int t = 0; t < T; t++) {
        int64_t best = -1;
        uint64_t bi = 0;
        for (uint64_t i = 0; i < nc; i++) {
            if (taken[i]) continue;
            int64_t r = (int64_t)c[i].occ * (int64_t)((int)c[i].len - overlap[i]);
            if (best < 0 || r > best) {
                best = r;
                bi = i;
            } else if (r == best) {
                if (c[i].len > c[bi].len) {
                    bi = i;
                } else if (c[i].len == c[bi].len) {
                    unpack(c[i].key, (int)c[i].len, a);
                    unpack(c[bi].key, (int)c[bi].len, b);
                    if (memcmp(a, b, c[i].len) < 0) bi = i;
                }
            }
        }
        if (best <= 0) break;
        taken[bi] = 1;
        unpack(c[bi].key, (int)c[bi].len, pat + 8 * chosen);
        pat_len[chosen] = (uint8_t)c[bi].len;
        chosen++;
        unpack(c[bi].key, (int)c[bi].len, b);
        for (uint64_t i = 0; i < nc; i++) {
            if (taken[i] || overlap[i] >= (int)c[i].len) continue;
            unpack(c[i].key, (int)c[i].len, a);
            int l = lcs_len(a, (int)c[i].len, b, (int)c[bi].len);
            if (l > overlap[i]) overlap[i] = l;
        }
    }
    free(c);
    free(overlap);
    free(taken);
    return chosen;
}
